"""Bounds audit, on the CPU, of the generic matching kernel that serves GRID blocks (the
paper's far path, Sec. 4.3.4 "Far Objects"): the kernel's index arithmetic restated
(plan: clip, type, level box, GRID point grid; block: point rows and columns, template
and candidate reads, LDS cost slots, block slots) and run over every box of the GRID
parity inputs, asserting that every access the kernel makes without a guard lies in its
buffer and that every guarded one is guarded. No GPU."""
import numpy as np
import pytest

from paper_2604_07980_amd import synth

GRID_VARIANTS = {
    "grid_far": dict(tau_s=50, agg_mode=0,
                     far=dict(mode=1, bw=8, bh=8, n_side=8, dmin=0, dmax=15),
                     close=dict(mode=0, bw=8, bh=8, n_side=8, dmin=0, dmax=31)),
    "grid_both_s3": dict(tau_s=30, close_scale=3, min_point_pct=80,
                         far=dict(mode=1, bw=8, bh=8, n_side=5, dmin=1, dmax=9),
                         close=dict(mode=1, bw=8, bh=8, n_side=7, dmin=0, dmax=23)),
}


def _cdiv(a, s):
    return (a + s - 1) // s


def _plan(box, W, H, p):
    """The plan step's geometry of one box (None unless it is matched)."""
    x0, y0, x1, y1, flags = box
    cx0, cy0, cx1, cy1 = max(x0, 0), max(y0, 0), min(x1, W), min(y1, H)
    if not (flags & 1) or not (cx0 < cx1 and cy0 < cy1):
        return None
    far = max(cx1 - cx0, cy1 - cy0) < p["tau_s"]
    level = 0 if far else 1
    s = 1 if far else p["close_scale"]
    ph = p["far"] if far else p["close"]
    Ws, Hs = W // s, H // s
    lx0, lx1 = max(_cdiv(cx0, s), p["sx"]), min(_cdiv(cx1, s), Ws - p["sx"])
    ly0, ly1 = max(_cdiv(cy0, s), p["sy"]), min(_cdiv(cy1, s), Hs - p["sy"])
    if lx1 <= lx0 or ly1 <= ly0:
        return None
    lw, lh = lx1 - lx0, ly1 - ly0
    if ph["mode"] != 1:
        return None                       # TILED blocks are served by the other kernels
    nx, ny = min(ph["n_side"], lw), min(ph["n_side"], lh)
    dlo = ph["dmin"] // s
    nd = _cdiv(ph["dmax"] - ph["dmin"] + 1, s)
    return dict(level=level, s=s, Ws=Ws, Hs=Hs, lx0=lx0, ly0=ly0, lw=lw, lh=lh, nx=nx, ny=ny,
                dlo=dlo, nd=nd)


def _audit_block(g):
    """Every access of match_block_generic / generic_costs for one GRID block."""
    assert 1 <= g["nx"] <= 8 and 1 <= g["ny"] <= 8 and g["nx"] * g["ny"] <= 64
    assert 1 <= g["nd"] <= 256
    cols = [g["lx0"] + (2 * i + 1) * g["lw"] // (2 * g["nx"]) for i in range(g["nx"])]
    rows = [g["ly0"] + (2 * j + 1) * g["lh"] // (2 * g["ny"]) for j in range(g["ny"])]
    # rows index the level image without a guard; columns go through ld_word
    for y in rows:
        assert 0 <= y < g["Hs"]
    for x in cols:
        assert 0 <= x < g["Ws"]
    # LDS cost slots: kc = lane + 64 r < nd <= 256, two arrays of 256 entries
    for lane in range(64):
        for r in range(4):
            kc = lane + 64 * r
            if kc < g["nd"]:
                assert kc < 256
    # the winner and its neighbours read costf[max(best - 1, 0)], costf[min(best + 1, nd - 1)]
    for best in range(g["nd"]):
        assert 0 <= max(best - 1, 0) < 256 and 0 <= min(best + 1, g["nd"] - 1) < 256
    # occlusion: lane l tests point (l % nx, min(l / nx, ny - 1)), inside the grid
    for lane in range(64):
        pi, pj = lane % g["nx"], min(lane // g["nx"], g["ny"] - 1)
        assert 0 <= pi < g["nx"] and 0 <= pj < g["ny"]


@pytest.mark.parametrize("variant", list(GRID_VARIANTS))
@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_generic_kernel_indices_on_grid_inputs(variant, seed):
    p = synth.base_params()
    p.update({k: (dict(v) if isinstance(v, dict) else v) for k, v in GRID_VARIANTS[variant].items()})
    scenes = [synth.scene_small(1000 * seed + len(variant), H=120, W=200, n_planes=6),
              synth.scene_small(77 + len(variant), H=120, W=200, n_planes=6)]
    audited = 0
    for sc in scenes:
        H, W = sc.left.shape
        for b in sc.boxes.tolist():
            g = _plan(b, W, H, p)
            if g is None:
                continue
            _audit_block(g)
            audited += 1
    assert audited > 0


def test_generic_kernel_indices_extreme_grids():
    """GRID blocks at the edges of what the kernel takes: one-pixel level boxes, grids of
    8 x 8 over boxes narrower than 8 level px, 256 candidates, boxes at the image border."""
    p = synth.base_params()
    p.update(tau_s=1 << 30, far=dict(mode=1, bw=8, bh=8, n_side=8, dmin=0, dmax=255))
    W, H = 64, 48
    boxes = [[0, 0, W, H, 1], [3, 4, 4, 5, 1], [-10, -10, 5, 5, 1], [60, 40, 90, 90, 1],
             [10, 10, 14, 40, 1], [0, 0, 1, 1, 1]]
    n = 0
    for b in boxes:
        g = _plan(b, W, H, p)
        if g is not None:
            _audit_block(g)
            n += 1
    assert n >= 3
