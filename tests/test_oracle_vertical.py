"""Pins of the oracle's vertical offset search: the census cost equation of Sec. 4.3.2
over (dx, dy) offsets, the forward-backward check of Sec. 4.3.3 with a consistency test
on dx only. Pinned against facts fixed by construction: a texture moved by a known
(dx, dy) is found exactly with zero cost; a texture that varies along one axis only
makes the other offset a pure tie, which the tie order decides; the brute-force micro
oracle agrees block by block; and a zero vertical range is the horizontal search."""
import numpy as np
import pytest

from oracle import micro
from paper_2604_07980_amd import synth

H, W = 96, 160


def _params(dy_min, dy_max, **kw):
    p = synth.base_params()
    p.update(tau_s=48, dy_min=dy_min, dy_max=dy_max, lr_tol=0, min_point_pct=50)
    p["far"] = dict(mode=0, bw=4, bh=4, n_side=8, dmin=0, dmax=23)
    p["close"] = dict(mode=0, bw=8, bh=8, n_side=8, dmin=0, dmax=31)
    p.update(kw)
    return p


# two far boxes (side < 48) and one close box, apart (no occlusion), clear of the image
# border by more than the true offsets reach
BOXES = np.array([[20, 20, 50, 44, 1], [120, 56, 150, 80, 1], [56, 14, 112, 86, 1]], np.int32)


def _min_cost(blk, cf, k):
    return int(cf[k, :int(blk["nd"][k])].min())


def _run(orc, left, right, p):
    _, (res, blk, cf, cb, n) = orc.run_scene(left, right, p, BOXES, debug=True)
    return res, blk, cf, cb, n


@pytest.mark.parametrize("dx,dy,rng_", [(6, 2, (-3, 3)), (10, -4, (-4, 2)), (4, 0, (-2, 2)),
                                         (8, -2, (-2, -2))])
def test_known_2d_shift_is_found_exactly(orc, dx, dy, rng_):
    left, right = synth.shifted_texture(11, H, W, dx, dy)
    res, blk, cf, cb, n = _run(orc, left, right, _params(*rng_))
    el = blk["eligible"] == 1
    assert el.sum() > 20
    for k in np.flatnonzero(el):
        s = int(blk["level_scale"][k])
        assert blk["d_f"][k] == dx // s and blk["dy_f"][k] == dy // s, k
        assert cf[k, dx // s - blk["dlo"][k]] == 0          # zero cost at the truth
        assert blk["d_b"][k] == dx // s and blk["dy_b"][k] == dy // s
        assert blk["lr_ok"][k] == 1 and blk["valid"][k] == 1
        assert abs(float(blk["d_sub"][k]) - dx // s) <= 0.5
    assert (res["valid"] == 1).all()
    assert np.allclose(res["disparity"], dx, atol=1.0)   # half a level pixel at s = 2


def test_without_the_vertical_search_a_drift_is_missed(orc):
    """The same moved texture with dy = 0 only: the search cannot reach zero cost."""
    left, right = synth.shifted_texture(12, H, W, 6, 2)
    _, blk, cf, _, _ = _run(orc, left, right, _params(0, 0))
    el = blk["eligible"] == 1
    assert (blk["dy_f"][el] == 0).all()
    assert all(_min_cost(blk, cf, k) > 0 for k in np.flatnonzero(el))


def test_ties_along_dy_go_to_the_smallest_offset(orc):
    """Texture constant along y: every dy costs the same, so dy_f is the range start,
    while dx is still found."""
    left, right = synth.shifted_texture(13, H, W, 6, 0, mode="cols")
    _, blk, cf, _, _ = _run(orc, left, right, _params(-3, 2))
    el = blk["eligible"] == 1
    s = blk["level_scale"][el]
    assert (blk["d_f"][el] == 6 // s).all()
    assert (blk["dy_f"][el] == np.where(s == 1, -3, -2)).all()   # floor(-3 / s)
    assert (blk["dy_b"][el] == blk["dy_f"][el]).all()


def test_ties_along_dx_go_to_the_smallest_disparity(orc):
    """Texture constant along x: every d costs the same, so d_f is the range start,
    while dy is still found."""
    left, right = synth.shifted_texture(14, H, W, 0, -2, mode="rows")
    _, blk, _, _, _ = _run(orc, left, right, _params(-3, 3))
    el = blk["eligible"] == 1
    s = blk["level_scale"][el]
    assert (blk["d_f"][el] == blk["dlo"][el]).all()
    assert (blk["dy_f"][el] == -2 // s).all()


def test_level_range_covers_the_full_resolution_range(orc):
    """At scale s the level offsets run from floor(dy_min / s) to ceil(dy_max / s): a
    drift of -4 px lies outside [-3, 3] at s = 1 but its level value -2 lies inside
    [-2, 2] at s = 2."""
    left, right = synth.shifted_texture(15, H, W, 8, -4)
    _, blk, cf, _, _ = _run(orc, left, right, _params(-3, 3))
    el = blk["eligible"] == 1
    close = el & (blk["level_scale"] == 2)
    far = el & (blk["level_scale"] == 1)
    assert close.any() and far.any()
    assert (blk["dy_f"][close] == -2).all() and (blk["d_f"][close] == 4).all()
    assert all(_min_cost(blk, cf, k) > 0 for k in np.flatnonzero(far))


def test_zero_range_is_the_horizontal_search(orc):
    sc = synth.scene_small(21, H=H, W=W, n_planes=4)
    p0 = _params(0, 0)
    p1 = dict(p0)
    del p1["dy_min"], p1["dy_max"]
    r0 = orc.run_scene(sc.left, sc.right, p0, sc.boxes, debug=True)[1]
    r1 = orc.run_scene(sc.left, sc.right, p1, sc.boxes, debug=True)[1]
    for a, b in zip(r0[:4], r1[:4]):
        assert np.array_equal(a, b)
    assert (r0[1]["dy_f"] == 0).all() and (r0[1]["dy_b"] == 0).all()


@pytest.mark.parametrize("seed,dy", [(1, (-2, 1)), (2, (-1, 2)), (3, (0, 3))])
def test_vertical_search_vs_micro(orc, seed, dy):
    """Block by block against the brute-force micro oracle on a drifted scene."""
    p = _params(*dy)
    p["far"]["dmax"], p["close"]["dmax"] = 13, 23
    sc = synth.scene_small(300 + seed, H=64, W=104, n_planes=3)
    right = synth.drift_rows(sc.right, dy[0] + seed % 2)
    (L0, R0, L1, R1), (res, blk, cf, cb, n) = orc.run_scene(sc.left, right, p, sc.boxes, debug=True)
    s = p["close_scale"]
    mres, mblk, mtotal = micro.match_boxes({1: (L0, R0), s: (L1, R1)}, 104, 64, sc.boxes, p)
    assert mtotal == n
    for i, r in enumerate(mres):
        assert res["reason"][i] == r["reason"]
        assert res["disparity"][i] == np.float32(r["disparity"])
    for k, m in enumerate(mblk):
        assert int(blk["mask"][k]) == m["mask"] and blk["eligible"][k] == m["eligible"]
        if m["eligible"]:
            for f in ("d_f", "d_b", "dy_f", "dy_b", "lr_ok"):
                assert blk[f][k] == m[f], (k, f)
            assert blk["d_sub"][k] == np.float32(m["d_sub"])
            nd = int(blk["nd"][k])
            assert list(cf[k, :nd]) == m["cost_f"] and list(cb[k, :nd]) == m["cost_b"]
