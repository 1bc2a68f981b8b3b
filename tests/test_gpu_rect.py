"""Auto-rectification offset counts (Sec. 5.1) through the C ABI against the CPU oracle:
counts and checked disparity maps of every offset bit-exact, for several ROIs (at the
image edges too), windows and tolerances; the ground-like 1080p pair at the close level;
argument checks."""
import numpy as np
import pytest
import torch

from paper_2604_07980_amd import synth
from test_gpu_parity import _cuda

pytestmark = pytest.mark.gpu


def _desc(lib, left, right, s=1):
    L, R = _cuda(left), _cuda(right)
    g = lib.census_many([L, R], [s, s], 3, 4, 1)
    return g[0], g[1]


def _check(lib, orc, left, right, p, s=1):
    CLg, CRg = _desc(lib, left, right, s)
    counts, maps = lib.rect_offset_counts(CLg, CRg, p, with_maps=True)
    CL = CLg.cpu().numpy().view(np.uint64)
    CR = CRg.cpu().numpy().view(np.uint64)
    want, wmaps = orc.rect_counts(CL, CR, p, maps=True)
    assert (maps.cpu().numpy() == wmaps).all()
    assert (counts.cpu().numpy() == want).all()
    return want


CASES = [
    dict(roi_x0=20, roi_y0=30, roi_w=160, roi_h=60, delta_min=-4, delta_max=4, dmin=0, dmax=23,
         radius=2, lr_tol=1, d_min=2),
    dict(roi_x0=0, roi_y0=5, roi_w=200, roi_h=110, delta_min=0, delta_max=5, dmin=3, dmax=40,
         radius=1, lr_tol=0, d_min=0),                 # ROI at the left, right and top edges
    dict(roi_x0=77, roi_y0=64, roi_w=61, roi_h=53, delta_min=-3, delta_max=1, dmin=0, dmax=63,
         radius=3, lr_tol=2, d_min=5),                 # ragged sizes, bottom edge at -3
    dict(roi_x0=100, roi_y0=50, roi_w=1, roi_h=1, delta_min=-2, delta_max=2, dmin=0, dmax=15,
         radius=2, lr_tol=1, d_min=0),                 # one pixel
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("dy", [-2, 3])
def test_rect_counts_match_oracle(lib, orc, case, dy):
    left, right = synth.shifted_texture(60 + case, 120, 200, 7, dy)
    counts = _check(lib, orc, left, right, CASES[case])
    p = CASES[case]
    if case == 0:
        assert int(np.argmax(counts)) == dy - p["delta_min"]


def test_rect_drifted_scene(lib, orc):
    sc = synth.scene_small(77, H=160, W=256, n_planes=5)
    right = synth.drift_rows(sc.right, 2)
    p = dict(roi_x0=8, roi_y0=40, roi_w=240, roi_h=80, delta_min=-3, delta_max=3, dmin=0,
             dmax=31, radius=2, lr_tol=1, d_min=1)
    _check(lib, orc, sc.left, right, p)


def test_rect_road_pair_close_level(lib, orc):
    """The ground-like 1080p pair, right view 6 rows low, searched at scale 2 over a band
    of road rows; the library's filter then reports level offset 3."""
    left, right = synth.road_pair(drift=6)
    p = dict(roi_x0=0, roi_y0=300, roi_w=960, roi_h=128, delta_min=-4, delta_max=4, dmin=0,
             dmax=63, radius=2, lr_tol=1, d_min=2)
    counts = _check(lib, orc, left, right, p, s=2)
    f = lib.RectFilter(5, 1)
    assert f.update(counts, p["delta_min"]) == (3, 1)      # estimate 3, first step clamped


def test_rect_rejects_bad_arguments(lib):
    img = torch.zeros((64, 96), dtype=torch.uint8, device="cuda:0")
    CL, CR = lib.census_many([img, img], [1, 1])
    base = dict(roi_x0=10, roi_y0=20, roi_w=40, roi_h=20, delta_min=-2, delta_max=2, dmin=0,
                dmax=15, radius=2, lr_tol=1, d_min=0)
    bad = [dict(roi_y0=1), dict(roi_x0=60), dict(delta_min=3), dict(delta_min=-40, delta_max=40),
           dict(roi_w=0), dict(dmax=-1), dict(d_min=-1)]
    for b in bad:
        with pytest.raises((lib.OcsrError, ValueError)):
            lib.rect_offset_counts(CL, CR, dict(base, **b))
    with pytest.raises(lib.OcsrError) as e:
        lib.rect_offset_counts(CL, CR, dict(base, radius=4))
    assert e.value.code == lib.E_UNSUPPORTED


def test_rect_estimate_drives_the_vertical_offset(lib, orc):
    """The estimate feeds the matcher: the road pair's right view is 6 rows low; the
    offset search at s = 2 finds 3 level rows, i.e. 6 px, and ranging with dy fixed at
    6 px equals the oracle and validates nearly every block, where dy = 0 does not."""
    left, right = synth.road_pair(drift=6)
    p = dict(roi_x0=0, roi_y0=300, roi_w=960, roi_h=128, delta_min=-4, delta_max=4, dmin=0,
             dmax=63, radius=2, lr_tol=1, d_min=2)
    CLg, CRg = _desc(lib, left, right, 2)
    counts = lib.rect_offset_counts(CLg, CRg, p).cpu().numpy()
    raw, _ = lib.RectFilter(1, 100).update(counts, p["delta_min"])
    dy = 2 * raw
    assert dy == 6
    boxes = np.array([[100, 620, 260, 700, 1], [500, 700, 760, 820, 1], [900, 560, 960, 600, 1],
                      [1300, 800, 1700, 1000, 1], [1600, 600, 1650, 640, 1],
                      [300, 900, 700, 1060, 1]], np.int32)
    mp = synth.params_for(2)
    mp["dy_min"] = mp["dy_max"] = dy
    got = lib.results_to_numpy(lib.range_frame(_cuda(left), _cuda(right), _cuda(boxes), mp))
    want = orc.run_scene(left, right, mp, boxes)[1][0]
    from test_gpu_parity import assert_results_match
    assert_results_match(got, want)
    assert (got["n_valid"] >= 0.9 * got["n_blocks"]).all()
    plain = orc.run_scene(left, right, synth.params_for(2), boxes)[1][0]
    assert plain["n_valid"].sum() < 0.6 * got["n_valid"].sum()
