"""Brute-force cross-checks of the C oracle against the NumPy micro-oracle, and the
dense counterpart's pins. No GPU; tiny inputs only."""
import numpy as np
import pytest

from oracle import micro
from paper_2604_07980_amd import synth

VARIANTS = {
    "tiled_trim": dict(tau_s=40, far=dict(mode=0, bw=4, bh=4, n_side=8, dmin=0, dmax=15),
                       close=dict(mode=0, bw=8, bh=8, n_side=8, dmin=0, dmax=31)),
    "tiled_seg_lr0": dict(tau_s=40, agg_mode=0, lr_tol=0,
                          far=dict(mode=0, bw=4, bh=2, n_side=8, dmin=2, dmax=13),
                          close=dict(mode=0, bw=6, bh=5, n_side=8, dmin=3, dmax=28)),
    "grid_far": dict(tau_s=50, agg_mode=0,
                     far=dict(mode=1, bw=8, bh=8, n_side=8, dmin=0, dmax=15),
                     close=dict(mode=0, bw=8, bh=8, n_side=8, dmin=0, dmax=31)),
    "grid_both_s3": dict(tau_s=30, close_scale=3, min_point_pct=80,
                         far=dict(mode=1, bw=8, bh=8, n_side=5, dmin=1, dmax=9),
                         close=dict(mode=1, bw=8, bh=8, n_side=7, dmin=0, dmax=23)),
    "win5x5": dict(sx=2, sy=2, tau_s=40, trim_pct=10, n_min=2,
                   far=dict(mode=0, bw=3, bh=3, n_side=8, dmin=0, dmax=11),
                   close=dict(mode=0, bw=4, bh=4, n_side=8, dmin=0, dmax=19)),
}


def _params(v):
    p = synth.base_params()
    p.update({k: (dict(val) if isinstance(val, dict) else val) for k, val in VARIANTS[v].items()})
    return p


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_match_vs_micro(orc, variant, seed):
    p = _params(variant)
    sc = synth.scene_small(100 * seed + len(variant), H=72, W=112, n_planes=4)
    (L0, R0, L1, R1), (res, blk, cf, cb, n) = orc.run_scene(sc.left, sc.right, p, sc.boxes,
                                                            debug=True)
    s = p["close_scale"]
    lv = {1: (L0, R0), s: (L1, R1)}
    mres, mblk, mtotal = micro.match_boxes(lv, 112, 72, sc.boxes, p)
    assert mtotal == n
    for i, r in enumerate(mres):
        assert res["reason"][i] == r["reason"], (i, res[i], r)
        for f in ("valid", "n_blocks", "n_eligible", "n_valid", "n_used"):
            assert res[f][i] == r[f], (f, i)
        assert res["disparity"][i] == np.float32(r["disparity"])
        assert res["depth"][i] == np.float32(r["depth"])
    assert len(mblk) == n
    for b, m in zip(blk, mblk):
        for f in ("box", "u", "v", "px0", "py0", "nx", "ny", "mask", "eligible"):
            assert int(b[f]) == int(m[f]), f
        if m["eligible"]:
            assert b["d_f"] == m["d_f"] and b["d_b"] == m["d_b"] and b["lr_ok"] == m["lr_ok"]
            assert b["d_sub"] == np.float32(m["d_sub"])
    # cost volumes, block by block
    for k, m in enumerate(mblk):
        if m["eligible"]:
            nd = int(blk["nd"][k])
            assert list(cf[k, :nd]) == m["cost_f"]
            assert list(cb[k, :nd]) == m["cost_b"]


def test_match_edge_cases(orc):
    """Boxes outside, partly outside, degenerate and thinner than a block."""
    sc = synth.scene_small(9, H=64, W=96, n_planes=2)
    p = _params("tiled_trim")
    boxes = np.array([[-30, -30, -1, -1, 1],    # fully outside: CLIPPED_EMPTY
                      [10, 10, 10, 40, 1],      # zero width
                      [90, 20, 140, 60, 1],     # partly outside
                      [0, 0, 96, 64, 1],        # whole image (close)
                      [20, 30, 23, 31, 1],      # thinner than the census margin rows
                      [40, 20, 46, 60, 0],      # not ranged
                      [5, 5, 12, 50, 1]],       # narrow: one shrunken column of blocks
                     np.int32)
    (L0, R0, L1, R1), (res, blk, cf, cb, n) = orc.run_scene(sc.left, sc.right, p, boxes, debug=True)
    mres, mblk, mtotal = micro.match_boxes({1: (L0, R0), 2: (L1, R1)}, 96, 64, boxes, p)
    assert [r["reason"] for r in mres] == list(res["reason"])
    assert res["reason"][0] == 2 and res["reason"][1] == 2 and res["reason"][5] == 1
    assert mtotal == n


def test_capacity_rules(orc):
    sc = synth.scene_small(4, H=64, W=96, n_planes=3)
    p = _params("tiled_trim")
    boxes = np.array([[0, 34, 96, 64, 1], [10, 5, 30, 25, 1], [50, 5, 62, 17, 1]], np.int32)
    _, (res0, *_rest) = orc.run_scene(sc.left, sc.right, p, boxes)
    nb = res0["n_blocks"]
    assert (nb > 0).all() and len(set(nb.tolist())) == 3
    cap = int(nb.max()) - 1
    _, (res, *_r) = orc.run_scene(sc.left, sc.right, dict(p, max_blocks_per_box=cap), boxes)
    big = nb > cap
    assert (res["reason"][big] == 7).all()
    assert (res["reason"][~big] == res0["reason"][~big]).all()
    # total capacity: blocks are numbered by a prefix over the boxes; a box whose range
    # passes the capacity is dropped
    _, (res3, *_r) = orc.run_scene(sc.left, sc.right, p, boxes, cap_blocks=int(nb[0] + nb[1]))
    assert res3["reason"][2] == 7
    assert (res3["reason"][:2] == res0["reason"][:2]).all()
    _, (res4, *_r) = orc.run_scene(sc.left, sc.right, p, boxes, cap_blocks=int(nb[0]) + 1)
    assert res4["reason"][1] == 7 and res4["reason"][2] == 7


# ------------------------------------------------------------------------------------
# dense counterpart
# ------------------------------------------------------------------------------------

@pytest.mark.parametrize("radius", [0, 1, 2])
@pytest.mark.parametrize("dr", [(0, 7), (2, 9)])
def test_dense_vs_micro(orc, radius, dr):
    sc = synth.scene_small(77, H=16, W=24, n_planes=2)
    CL = orc.census(sc.left, 2, 2, 1, 1)
    CR = orc.census(sc.right, 2, 2, 1, 1)
    a, ar = orc.dense(CL, CR, dr[0], dr[1], radius, 1)
    b, br = micro.dense(CL, CR, dr[0], dr[1], radius, 1)
    assert (a == b).all() and (ar == br).all()
    pts = np.array([[x, y] for y in range(16) for x in range(24)], np.int32)
    c = orc.dense_at(CL, CR, pts, dr[0], dr[1], radius, 1)
    assert (c == a.reshape(-1)).all()


def test_dense_integer_shift(orc):
    """R(x, y) = L(x + k, y): every pixel whose whole window sees the shifted texture has
    a zero-cost match at k, unique on the texture."""
    k = 9
    rng = np.random.default_rng(2)
    left = np.rint(synth.blurred_noise(rng, 40, 90)).astype(np.uint8)
    right = np.empty_like(left)
    right[:, :90 - k] = left[:, k:]
    right[:, 90 - k:] = rng.integers(0, 256, size=(40, k), dtype=np.uint8)
    CL = orc.census(left, 3, 4, 1, 1)
    CR = orc.census(right, 3, 4, 1, 1)
    d, _ = orc.dense(CL, CR, 0, 23, 2, 1)
    inner = d[6:34, 3 + k + 2 + 3: 90 - 3 - 2 - 3 - k]
    assert (inner == k).all()


def test_dense_mirror_symmetry(orc):
    """Mirroring both images and swapping them turns right-view matches into left-view
    ones: the Hamming distance is unchanged by the consistent bit permutation x -> -x.
    Holds wherever no window is clipped by the image side: x' in [r, W - 1 - r - dmax]."""
    sc = synth.scene_small(31, H=20, W=40, n_planes=2)
    CL = orc.census(sc.left, 2, 2, 1, 1)
    CR = orc.census(sc.right, 2, 2, 1, 1)
    _, dr = orc.dense(CL, CR, 0, 11, 2, 1)
    FL = orc.census(np.ascontiguousarray(sc.right[:, ::-1]), 2, 2, 1, 1)
    FR = orc.census(np.ascontiguousarray(sc.left[:, ::-1]), 2, 2, 1, 1)
    vol = micro.dense_volume(FL, FR, 0, 11, 2)
    dl_mirror = np.argmin(vol, axis=0)
    cols = slice(2, 40 - 1 - 2 - 11 + 1)
    assert (dl_mirror[:, ::-1][:, cols] == dr[:, cols]).all()


def test_sparse_is_sum_of_dense(orc):
    """A full-mask block's forward cost S_f(d) is the sum of the per-pixel (radius 0)
    dense costs over its points: ties the sparse path to the dense one."""
    sc = synth.scene_small(12, H=48, W=80, n_planes=1)
    p = _params("tiled_trim")
    boxes = np.array([[30, 10, 60, 40, 1]], np.int32)
    (L0, R0, _, _), (res, blk, cf, cb, n) = orc.run_scene(sc.left, sc.right, p, boxes, debug=True)
    vol = micro.dense_volume(L0, R0, 0, 15, 0)
    for k, b in enumerate(blk):
        if not b["eligible"] or int(b["mask"]) != (1 << int(b["nx"] * b["ny"])) - 1:
            continue
        ys = slice(b["py0"], b["py0"] + b["ny"])
        xs = slice(b["px0"], b["px0"] + b["nx"])
        want = vol[:, ys, xs].sum(axis=(1, 2))
        assert list(cf[k, :16]) == list(want)
