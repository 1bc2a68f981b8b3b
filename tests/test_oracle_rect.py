"""Pins of the oracle's auto-rectification offset (Sec. 5.1): the offset search finds a
vertical misalignment built into the pair; moving the descriptors equals moving the image
away from its border (the census is translation invariant there); the temporal filter
follows hand-worked sequences; the tie rule of the estimate."""
import numpy as np
import pytest

from paper_2604_07980_amd import synth

H, W = 120, 200


def _rect(**kw):
    p = dict(roi_x0=20, roi_y0=30, roi_w=160, roi_h=60, delta_min=-4, delta_max=4,
             dmin=0, dmax=23, radius=2, lr_tol=1, d_min=0)
    p.update(kw)
    return p


@pytest.mark.parametrize("dy", [-3, 0, 2, 4])
def test_offset_of_a_misaligned_pair_is_found(orc, dy):
    """right(x - 7, y + dy) = left(x, y): moving the left image down by dy aligns the
    pair, so the count peaks there; the blurred texture still half-matches one row off,
    but offsets two or more rows away fall well below."""
    left, right = synth.shifted_texture(50 + dy, H, W, 7, dy)
    CL, CR = orc.census(left, 3, 4, 1, 1), orc.census(right, 3, 4, 1, 1)
    p = _rect(d_min=2)
    counts = orc.rect_counts(CL, CR, p)
    k = dy - p["delta_min"]
    assert int(np.argmax(counts)) == k and (np.delete(counts, k) < counts[k]).all()
    assert counts[k] > 0.9 * p["roi_w"] * p["roi_h"] - 7 * p["roi_h"]
    far = np.abs(np.arange(len(counts)) + p["delta_min"] - dy) >= 2
    assert counts[far].max() < 0.75 * counts[k]
    raw, _ = orc.rect_filter(counts[None, :], p["delta_min"], 1, 100)
    assert raw[0] == dy


def test_moving_descriptors_equals_moving_the_image(orc):
    """Left image moved down by delta (cut from a taller texture, so nothing is padded):
    its census over the ROI equals the original census moved, and so do the maps."""
    rng = np.random.default_rng(5)
    big = np.rint(synth.blurred_noise(rng, H + 20, W)).astype(np.uint8)
    left = big[10:10 + H]
    right = np.ascontiguousarray(np.roll(left, -5, axis=1))
    CL, CR = orc.census(left, 3, 4, 1, 1), orc.census(right, 3, 4, 1, 1)
    p = _rect(delta_min=-3, delta_max=3)
    counts, maps = orc.rect_counts(CL, CR, p, maps=True)
    for delta in range(-3, 4):
        moved = big[10 - delta:10 - delta + H]               # row y is left row y - delta
        CLm = orc.census(np.ascontiguousarray(moved), 3, 4, 1, 1)
        q = dict(p, delta_min=0, delta_max=0)
        c1, m1 = orc.rect_counts(CLm, CR, q, maps=True)
        assert c1[0] == counts[delta + 3]
        assert (m1[0] == maps[delta + 3]).all()


def test_filter_hand_sequence(orc):
    """window 3, max_step 1, offsets -1..1. Estimates 0, 1, 1, -1, 0 (the last a
    three-way tie, which goes to 0); medians 0, 0 (lower middle of 0, 1), 1, 1, 0;
    outputs 0, 0, 1, 1, 0."""
    seq = [[0, 5, 1], [0, 0, 9], [0, 0, 9], [9, 0, 0], [1, 1, 1]]
    raw, filt = orc.rect_filter(seq, -1, 3, 1)
    assert raw.tolist() == [0, 1, 1, -1, 0]
    assert filt.tolist() == [0, 0, 1, 1, 0]


def test_filter_step_is_clamped(orc):
    """A jump of the estimate from 0 to 5 is followed 2 per frame once the median moves."""
    seq = [[0] * 5 + [9] + [0] * 5] * 1 + [[0] * 10 + [9]] * 6   # offsets -5..5
    raw, filt = orc.rect_filter(seq, -5, 3, 2)
    assert raw.tolist() == [0] + [5] * 6
    # medians: 0, 0 (lower of 0, 5), 5, 5, ...; outputs step by 2
    assert filt.tolist() == [0, 0, 2, 4, 5, 5, 5]


def test_estimate_ties(orc):
    raw, _ = orc.rect_filter([[3, 3, 3, 3, 3]], -2, 1, 10)
    assert raw[0] == 0                    # nearest zero
    raw, _ = orc.rect_filter([[7, 1, 1, 7, 0]], -2, 1, 10)   # -2 and 1 tie; |1| < |-2|
    assert raw[0] == 1
    raw, _ = orc.rect_filter([[0, 7, 1, 7, 0]], -2, 1, 10)   # -1 and 1 tie: the lower
    assert raw[0] == -1


def test_roi_leaving_the_image_is_rejected(orc):
    CL = np.zeros((H, W), np.uint64)
    with pytest.raises(ValueError):
        orc.rect_counts(CL, CL, _rect(roi_y0=2, delta_max=3))


def test_road_pair_drift_at_the_close_level(orc):
    """The ground-like pair with its right view 6 rows low: at scale 2 the search over a
    band of road rows finds 3 level rows."""
    left, right = synth.road_pair(drift=6)
    CL, CR = orc.census(left, 3, 4, 2, 1), orc.census(right, 3, 4, 2, 1)
    p = dict(roi_x0=0, roi_y0=300, roi_w=960, roi_h=128, delta_min=-4, delta_max=4, dmin=0,
             dmax=63, radius=2, lr_tol=1, d_min=2)
    counts = orc.rect_counts(CL, CR, p)
    raw, _ = orc.rect_filter(counts[None, :], p["delta_min"], 1, 10)
    assert raw[0] == 3
