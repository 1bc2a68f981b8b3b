"""The census-tile rule of whole-frame calls, checked on the CPU against the oracle's own
searches: every descriptor the oracle's forward and backward searches read lies in a
tile the rule makes, and boxes of no search make no tile."""
import numpy as np
import pytest

from paper_2604_07980_amd import accounting, synth
from test_gpu_parity import _params

TX, TY = accounting.TILE_X, accounting.TILE_Y


def _read_tiles(blk, W, H, p):
    """Tiles holding a descriptor some eligible block's searches read (forward: template
    CL(x, y) and CR(x - d, y + e); backward: CR(x - d_f, y + e_f) and
    CL(x - d_f + d, y + e_f - e); d and e over the level candidates; reads outside the
    level image are not reads)."""
    s = p["close_scale"]
    out = set()
    for b in blk[blk["eligible"] == 1]:
        level = 0 if b["level_scale"] == 1 else 1
        sl = 1 if level == 0 else s
        Wl, Hl = (W, H) if level == 0 else (W // s, H // s)
        dlo, nd = int(b["dlo"]), int(b["nd"])
        dhi = dlo + nd - 1
        eylo, eyhi = p.get("dy_min", 0) // sl, -(-p.get("dy_max", 0) // sl)
        x0, nx, y0, ny, d_f = int(b["px0"]), int(b["nx"]), int(b["py0"]), int(b["ny"]), int(b["d_f"])
        e_f = int(b["dy_f"])
        # (view, x range, y range) of each read
        ranges = [(0, x0, x0 + nx, y0, y0 + ny),
                  (1, x0 - dhi, x0 - dlo + nx, y0 + eylo, y0 + ny + eyhi),
                  (1, x0 - d_f, x0 - d_f + nx, y0 + e_f, y0 + e_f + ny),
                  (0, x0 - d_f + dlo, x0 - d_f + dhi + nx, y0 + e_f - eyhi, y0 + e_f - eylo + ny)]
        for view, a, e, ya, yb in ranges:
            a, e, ya, yb = max(a, 0), min(e, Wl), max(ya, 0), min(yb, Hl)
            if a >= e or ya >= yb:
                continue
            for ty in range(ya // TY, (yb - 1) // TY + 1):
                for tx in range(a // TX, (e - 1) // TX + 1):
                    out.add((level, view, tx, ty))
    return out


@pytest.mark.parametrize("variant", ["tiled_trim", "tiled_seg_lr0", "wide_range", "win5x5"])
@pytest.mark.parametrize("seed", [3, 4])
def test_rule_covers_every_read(orc, variant, seed):
    p = _params(variant)
    sc = synth.scene_small(300 + seed, H=180, W=320, n_planes=6)
    _, (res, blk, _, _, n) = orc.run_scene(sc.left, sc.right, p, sc.boxes, debug=True)
    H, W = sc.left.shape
    rule = accounting.census_tiles(W, H, sc.boxes, p)
    read = _read_tiles(blk[:n], W, H, p)
    assert read, "some block searched"
    assert read <= rule, sorted(read - rule)[:5]


@pytest.mark.parametrize("shift", [5, 70, 150])
def test_rule_covers_reads_at_large_disparity(orc, shift):
    """A pair shifted by `shift` pixels, so that the winners (and the backward searches
    around them) sit far from the box; boxes straddle tile borders at both levels."""
    rng = np.random.default_rng(shift)
    H, W = 256, 640
    left = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    right = np.roll(left, -shift, axis=1)
    p = synth.params_for(2)
    p["far"]["dmax"], p["close"]["dmax"] = 191, 255
    boxes = np.array([[300, 20, 340, 60, 1], [380, 100, 410, 130, 1], [250, 140, 380, 250, 1],
                      [500, 30, 620, 200, 1], [W - 30, 5, W, 30, 1]], np.int32)
    _, (res, blk, _, _, n) = orc.run_scene(left, right, p, boxes, debug=True)
    rule = accounting.census_tiles(W, H, boxes, p)
    read = _read_tiles(blk[:n], W, H, p)
    assert read <= rule, sorted(read - rule)[:5]


def test_rule_covers_reads_of_the_realistic_frame(orc):
    p = synth.params_for(2)
    sc = synth.scene_realistic()
    _, (res, blk, _, _, n) = orc.run_scene(sc.left, sc.right, p, sc.boxes, debug=True)
    rule = accounting.census_tiles(1920, 1080, sc.boxes, p)
    read = _read_tiles(blk[:n], 1920, 1080, p)
    assert read <= rule, sorted(read - rule)[:5]


@pytest.mark.parametrize("scale", [2, 3])
@pytest.mark.parametrize("dy", [(-3, 3), (-6, -2), (1, 5)])
def test_rule_covers_vertical_reads(orc, dy, scale):
    """With a vertical range the searches read rows above and below the box: boxes along
    tile rows and the image's top and bottom edges, right view drifted."""
    rng = np.random.default_rng(40 + dy[0])
    H, W = 200, 400
    left = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    right = synth.drift_rows(np.roll(left, -9, axis=1), dy[1] - 1)
    p = synth.params_for(2)
    p["far"]["dmax"], p["close"]["dmax"] = 31, 63
    p["dy_min"], p["dy_max"] = dy
    p["close_scale"] = scale
    boxes = np.array([[40, 0, 70, 28, 1], [100, 26, 130, 40, 1], [150, 60, 260, 130, 1],
                      [300, 150, 340, 200, 1], [20, 120, 120, 200, 1], [330, 30, 390, 62, 1]],
                     np.int32)
    _, (res, blk, _, _, n) = orc.run_scene(left, right, p, boxes, debug=True)
    rule = accounting.census_tiles(W, H, boxes, p)
    read = _read_tiles(blk[:n], W, H, p)
    assert read <= rule, sorted(read - rule)[:5]
    # the vertical range moves the rows read (a range of one sign moves the right view's
    # rows away from the box's own)
    p0 = dict(p, dy_min=0, dy_max=0)
    assert accounting.census_tiles(W, H, boxes, p0) != rule


def test_rule_without_ranged_boxes_is_empty():
    p = synth.params_for(2)
    sc = synth.scene_realistic()
    boxes = sc.boxes.copy()
    boxes[:, 4] = 0
    assert accounting.census_tiles(1920, 1080, boxes, p) == set()


def test_full_rule_and_pixels():
    p = synth.params_for(2)
    full = accounting.census_tiles(1920, 1080, np.zeros((0, 5), np.int32), p, full=True)
    # 30 x 34 tiles per view at 1920x1080, 15 x 17 at 960x540
    assert len(full) == 2 * 30 * 34 + 2 * 15 * 17
    assert accounting.census_pixels(1920, 1080, full, p) == 2 * 1920 * 1080 + 2 * 960 * 540


def test_realistic_frame_makes_a_fraction():
    p = synth.params_for(2)
    sc = synth.scene_realistic()
    made = accounting.census_tiles(1920, 1080, sc.boxes, p)
    assert 0.05 < accounting.census_pixels(1920, 1080, made, p) / (2 * 1920 * 1080 + 2 * 960 * 540) < 0.5
