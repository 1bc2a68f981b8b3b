"""Vertical offset search (census cost over (dx, dy), Sec. 4.3.2) through the C ABI
against the CPU oracle: block tables, winners (d and dy, both directions), masks and
cost rows bit-exact, sub-pixel disparity and depth within the parity tolerances. Inputs
are the seeded scenes of the other parity tests with the right view moved by a few rows
(a residual vertical misalignment of the rectified pair), and a texture moved by a known
(dx, dy)."""
import numpy as np
import pytest
import torch

from paper_2604_07980_amd import synth
from test_gpu_parity import (_check_debug, _cuda, _gpu_levels, _params, assert_results_match,
                             lib_options)

pytestmark = pytest.mark.gpu

TILED = ("tiled_trim", "tiled_seg_lr0", "win5x5")


# small boxes added to every drifted scene so that both levels have blocks
FAR_BOXES = np.array([[150, 86, 176, 110, 1], [12, 96, 36, 116, 1], [100, 8, 120, 30, 1]], np.int32)


def _drifted(seed, H, W, n_planes, drift):
    sc = synth.scene_small(seed, H=H, W=W, n_planes=n_planes)
    boxes = np.concatenate([sc.boxes.reshape(-1, 5), FAR_BOXES]).astype(np.int32)
    return synth.Scene(sc.left, synth.drift_rows(sc.right, drift), boxes, sc.truth, sc.seed)


def _with_dy(p, lo, hi):
    p = dict(p)
    p["dy_min"], p["dy_max"] = lo, hi
    return p


@pytest.mark.parametrize("variant", TILED)
@pytest.mark.parametrize("dy", [(-2, 2), (-3, 1), (0, 3), (-1, -1), (2, 2)])
def test_vertical_match_parity(lib, orc, variant, dy):
    p = _with_dy(_params(variant), *dy)
    p["tau_s"] = 40
    sc = _drifted(700 + 31 * dy[0] + dy[1] + len(variant), 120, 200, 8, dy[0] + 1)
    (L0, R0, L1, R1), (res, blk, cf, cb, n) = orc.run_scene(sc.left, sc.right, p, sc.boxes,
                                                            debug=True)
    assert (blk["level_scale"] == 1).any() and (blk["level_scale"] > 1).any()   # both levels
    g = _gpu_levels(lib, sc.left, sc.right, p)
    out, extra = lib.match_boxes(*g, _cuda(sc.boxes), p, debug=True, cap_blocks=max(n, 1) + 5)
    assert_results_match(lib.results_to_numpy(out), res)
    _check_debug(lib, extra, blk, cf, cb, n)


def test_vertical_known_shift_is_exact(lib, orc):
    """A texture moved by (6, 2): every eligible block finds d = 6 / s, dy = 2 / s."""
    H, W = 96, 160
    left, right = synth.shifted_texture(11, H, W, 6, 2)
    boxes = np.array([[20, 20, 50, 44, 1], [120, 56, 150, 80, 1], [56, 14, 112, 86, 1]], np.int32)
    p = _with_dy(synth.base_params(), -3, 3)
    p.update(tau_s=48, lr_tol=0)
    p["far"] = dict(mode=0, bw=4, bh=4, n_side=8, dmin=0, dmax=23)
    p["close"] = dict(mode=0, bw=8, bh=8, n_side=8, dmin=0, dmax=31)
    _, (res, blk, cf, cb, n) = orc.run_scene(left, right, p, boxes, debug=True)
    g = _gpu_levels(lib, left, right, p)
    out, extra = lib.match_boxes(*g, _cuda(boxes), p, debug=True, cap_blocks=n)
    _, rec, _, _ = lib.debug_to_numpy(extra)
    el = rec["eligible"] == 1
    s = rec["level_scale"][el]
    assert el.sum() > 20
    assert (rec["d_f"][el] == 6 // s).all() and (rec["dy_f"][el] == 2 // s).all()
    assert (rec["d_b"][el] == rec["d_f"][el]).all() and (rec["dy_b"][el] == rec["dy_f"][el]).all()
    assert_results_match(lib.results_to_numpy(out), res)
    _check_debug(lib, extra, blk, cf, cb, n)


def test_vertical_realistic_frame(lib, orc):
    """The 1080p benchmark frame with its right view 2 rows low, dy in [-3, 3]: whole
    frame (census of the tiles the widened searches read, then matching), against the
    oracle's full-image census path; the result must not depend on the census option,
    nor on the fused option (a vertical range always takes the multi-launch path)."""
    sc = synth.scene_realistic()
    sc = synth.Scene(sc.left, synth.drift_rows(sc.right, 2), sc.boxes, sc.truth, sc.seed)
    p = _with_dy(synth.params_for(2), -3, 3)
    _, (res, *_r) = orc.run_scene(sc.left, sc.right, p, sc.boxes)
    outs = []
    for full in (0, 1):
        for fused in (False, True):
            lib.set_option(lib.OPTION_FULL_CENSUS, full)
            try:
                with lib_options(lib, fused=fused):
                    got = lib.results_to_numpy(lib.range_frame(_cuda(sc.left), _cuda(sc.right),
                                                               _cuda(sc.boxes), p))
            finally:
                lib.set_option(lib.OPTION_FULL_CENSUS, 0)
            assert_results_match(got, res)
            outs.append(got.view(np.int32))
    for o in outs[1:]:
        assert (o == outs[0]).all()
    assert res["valid"][:32].sum() >= 20
    # without the vertical search the same drifted frame ranges worse
    _, (res0, *_r) = orc.run_scene(sc.left, sc.right, synth.params_for(2), sc.boxes)
    assert res["n_valid"].sum() > res0["n_valid"].sum()


def test_vertical_batch_and_graph(lib, orc):
    """Several drifted frames in one batch call, then the same call replayed from a HIP
    graph three times, each against the oracle."""
    p = _with_dy(synth.base_params(), -2, 2)
    p["tau_s"] = 40
    p["far"].update(dmax=15)
    p["close"].update(dmax=63)
    scenes = [_drifted(1500 + k, 160, 224, 3 + 2 * k, k - 1) for k in range(4)]
    want = np.concatenate([orc.run_scene(sc.left, sc.right, p, sc.boxes)[1][0] for sc in scenes])
    frames = [(_cuda(sc.left), _cuda(sc.right), len(sc.boxes)) for sc in scenes]
    boxes = _cuda(np.concatenate([sc.boxes for sc in scenes]).astype(np.int32))
    got = lib.results_to_numpy(lib.range_batch(frames, boxes, p))
    assert_results_match(got, want)
    with lib_options(lib, graph=True):
        for _ in range(3):
            g = lib.results_to_numpy(lib.range_batch(frames, boxes, p))
            torch.cuda.synchronize()
            assert (g.view(np.int32) == got.view(np.int32)).all()


def test_vertical_zero_range_matches_horizontal_kernels(lib):
    """dy_min = dy_max = 0 keeps the horizontal kernels: identical results and records."""
    p = _params("tiled_trim")
    sc = synth.scene_small(4242, H=120, W=200, n_planes=6)
    g = _gpu_levels(lib, sc.left, sc.right, p)
    a, ea = lib.match_boxes(*g, _cuda(sc.boxes), p, debug=True, cap_blocks=4096)
    b, eb = lib.match_boxes(*g, _cuda(sc.boxes), _with_dy(p, 0, 0), debug=True, cap_blocks=4096)
    assert (a.cpu().numpy() == b.cpu().numpy()).all()
    ra, rb = lib.debug_to_numpy(ea)[1], lib.debug_to_numpy(eb)[1]
    assert (ra.view(np.uint8) == rb.view(np.uint8)).all()
    assert (ra["dy_f"] == 0).all() and (ra["dy_b"] == 0).all()


def test_vertical_rejected_arguments(lib):
    """Bad or oversized vertical ranges fail on the host before any launch."""
    img = torch.zeros((64, 96), dtype=torch.uint8, device="cuda:0")
    g = lib.census_many([img, img, img, img], [1, 1, 2, 2])
    boxes = torch.tensor([[10, 10, 40, 40, 1]], dtype=torch.int32, device="cuda:0")
    base = _params("tiled_trim")
    cases = [((3, 2), lib.E_INVALID, base),
             ((-33, 0), lib.E_INVALID, base),
             ((0, 33), lib.E_INVALID, base),
             ((-8, 8), lib.E_UNSUPPORTED, _params("wide_range")),    # LDS / candidate limit
             ((-32, 32), lib.E_UNSUPPORTED, synth.base_params())]    # 32 x 65 > 2048 candidates
    for (lo, hi), code, p in cases:
        with pytest.raises(lib.OcsrError) as e:
            lib.match_boxes(*g, boxes, _with_dy(p, lo, hi))
        assert e.value.code == code, (lo, hi)
    # the stated limit of an 8 x 8 path with 96 candidates: 21 level offsets run (dy +-20
    # at s = 2), 23 do not
    out = lib.match_boxes(*g, boxes, _with_dy(synth.base_params(), -20, 20))
    assert out.shape == (1, 8)
    with pytest.raises(lib.OcsrError) as e:
        lib.match_boxes(*g, boxes, _with_dy(synth.base_params(), -22, 22))
    assert e.value.code == lib.E_UNSUPPORTED


@pytest.mark.parametrize("dy", [(-3, 3), (0, 4)])
def test_vertical_ring_path_records(lib, orc, dy):
    """Long strips (96 close candidates at s = 2) take the ring of strip rows rather than
    staging every row at once: block records and cost rows against the oracle."""
    p = _with_dy(synth.params_for(2), *dy)
    p["tau_s"] = 40
    sc = _drifted(2200 + dy[0], 200, 320, 6, dy[0] + 2)
    (L0, R0, L1, R1), (res, blk, cf, cb, n) = orc.run_scene(sc.left, sc.right, p, sc.boxes,
                                                            debug=True)
    assert (blk["nd"][blk["level_scale"] == 2] == 96).all() and (blk["level_scale"] == 2).any()
    g = _gpu_levels(lib, sc.left, sc.right, p)
    out, extra = lib.match_boxes(*g, _cuda(sc.boxes), p, debug=True, cap_blocks=max(n, 1))
    assert_results_match(lib.results_to_numpy(out), res)
    _check_debug(lib, extra, blk, cf, cb, n)


@pytest.mark.parametrize("dy", [(-4, 2), (1, 5)])
def test_vertical_close_scale_3(lib, orc, dy):
    """Close level at scale 3: level offsets floor(dy_min / 3) .. ceil(dy_max / 3)."""
    p = _with_dy(_params("tiled_trim"), *dy)
    p.update(close_scale=3, tau_s=40)
    sc = _drifted(2300 + dy[0], 150, 240, 6, dy[1])
    (L0, R0, L1, R1), (res, blk, cf, cb, n) = orc.run_scene(sc.left, sc.right, p, sc.boxes,
                                                            debug=True)
    assert (blk["level_scale"] == 3).any()
    s = 3
    g = lib.census_many([_cuda(sc.left), _cuda(sc.right), _cuda(sc.left), _cuda(sc.right)],
                        [1, 1, s, s], p["sx"], p["sy"], p["sentinel"])
    out, extra = lib.match_boxes(*g, _cuda(sc.boxes), p, debug=True, cap_blocks=max(n, 1))
    assert_results_match(lib.results_to_numpy(out), res)
    _check_debug(lib, extra, blk, cf, cb, n)
    got = lib.results_to_numpy(lib.range_frame(_cuda(sc.left), _cuda(sc.right), _cuda(sc.boxes), p))
    assert_results_match(got, res)


@pytest.mark.parametrize("seed", range(8))
def test_vertical_random_cases(lib, orc, seed):
    """Seeded random path shapes, ranges, drifts and scales, block records included."""
    rng = np.random.default_rng(4000 + seed)
    variant = TILED[seed % len(TILED)]
    lo = int(rng.integers(-6, 4))
    hi = lo + int(rng.integers(0, 7))
    p = _with_dy(_params(variant), lo, hi)
    p["tau_s"] = int(rng.integers(24, 64))
    p["close_scale"] = int(rng.choice([2, 3]))
    p["close"] = dict(p["close"], dmax=int(rng.integers(p["close"]["dmin"] + 4, 120)))
    H, W = int(rng.integers(96, 200)), int(rng.integers(128, 320))
    sc = _drifted(4100 + seed, H, W, int(rng.integers(2, 9)), int(rng.integers(-4, 5)))
    (L0, R0, L1, R1), (res, blk, cf, cb, n) = orc.run_scene(sc.left, sc.right, p, sc.boxes,
                                                            debug=True)
    s = p["close_scale"]
    g = lib.census_many([_cuda(sc.left), _cuda(sc.right), _cuda(sc.left), _cuda(sc.right)],
                        [1, 1, s, s], p["sx"], p["sy"], p["sentinel"])
    out, extra = lib.match_boxes(*g, _cuda(sc.boxes), p, debug=True, cap_blocks=max(n, 1))
    assert_results_match(lib.results_to_numpy(out), res)
    _check_debug(lib, extra, blk, cf, cb, n)
    got = lib.results_to_numpy(lib.range_frame(_cuda(sc.left), _cuda(sc.right), _cuda(sc.boxes), p))
    assert_results_match(got, res)
