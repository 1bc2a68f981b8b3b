"""Pins of the oracle's priority object selection (Sec. 4.3.5, last sentence: over the
budget, the objects in a central crop take precedence, then the nearest others). The
paper gives no example, so the pins are a hand-worked frame, the special cases that fix
the order by a library sort or make the selection the identity, and invariants of the
rule."""
import numpy as np
import pytest

W, H = 1000, 600
CROP = (333, 0, 667, 1000)      # x in [333, 667), full height


def _hand_boxes():
    return np.array([
        [400, 200, 500, 300, 1],    # 0 A: frontal, bottom 300
        [450, 400, 550, 500, 1],    # 1 B: frontal, bottom 500
        [0, 500, 100, 590, 1],      # 2 C: side, bottom 590
        [800, 300, 900, 400, 1],    # 3 D: side, bottom 400
        [420, 100, 480, 560, 0],    # 4 E: not ranged
        [-50, 10, -10, 50, 1],      # 5 F: clipped empty
        [350, 450, 420, 500, 1],    # 6 G: frontal, bottom 500 (ties B, larger index)
    ], np.int32)


def test_hand_worked_frame(orc):
    boxes = _hand_boxes()
    out, rank = orc.select_boxes(boxes, W, H, 3, CROP)
    # order: B, G (frontal, bottom 500, by index), A (frontal, 300), C (590), D (400)
    assert rank.tolist() == [2, 0, 3, 4, -1, -1, 1]
    assert out[:, 4].tolist() == [1, 1, 0, 0, 0, 1, 1]
    assert (out[:, :4] == boxes[:, :4]).all()


def test_budget_at_or_above_the_count_keeps_every_box(orc):
    boxes = _hand_boxes()
    for k in (5, 6, 1000):
        out, rank = orc.select_boxes(boxes, W, H, k, CROP)
        assert (out == boxes).all()
        assert sorted(rank[rank >= 0].tolist()) == list(range(5))


def test_zero_budget_ranges_nothing(orc):
    out, rank = orc.select_boxes(_hand_boxes(), W, H, 0, CROP)
    # every candidate loses the flag; the clipped-empty box is no candidate and keeps it
    assert out[:, 4].tolist() == [0, 0, 0, 0, 0, 1, 0]
    assert (rank[[4, 5]] == -1).all()


def test_whole_frame_crop_is_a_sort_by_bottom(orc):
    """With the crop covering the frame every candidate is frontal, so the order is the
    library sort by descending clipped bottom, then index."""
    rng = np.random.default_rng(3)
    n = 300
    x0 = rng.integers(-50, W, n)
    y0 = rng.integers(-50, H, n)
    boxes = np.stack([x0, y0, x0 + rng.integers(1, 200, n), y0 + rng.integers(1, 200, n),
                      np.ones(n, int)], 1).astype(np.int32)
    out, rank = orc.select_boxes(boxes, W, H, 40, (0, 0, 1000, 1000))
    cand = (np.minimum(boxes[:, 2], W) > np.maximum(boxes[:, 0], 0)) & \
           (np.minimum(boxes[:, 3], H) > np.maximum(boxes[:, 1], 0))
    idx = np.flatnonzero(cand)
    bottom = np.minimum(boxes[idx, 3], H)
    order = idx[np.lexsort((idx, -bottom))]
    assert (rank[order] == np.arange(len(order))).all()
    assert (rank[~cand] == -1).all()
    assert set(np.flatnonzero((out[:, 4] & 1).astype(bool) & cand)) == set(order[:40])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_frontal_before_proximity(orc, seed):
    """Invariants: a kept side box means every frontal box is kept; within each class the
    kept boxes are the nearest; boxes that are not candidates never change."""
    rng = np.random.default_rng(seed)
    n = 200
    x0 = rng.integers(-80, W, n)
    y0 = rng.integers(-80, H, n)
    boxes = np.stack([x0, y0, x0 + rng.integers(1, 300, n), y0 + rng.integers(1, 200, n),
                      rng.integers(0, 3, n) > 0], 1).astype(np.int32)
    k = int(rng.integers(5, 60))
    out, rank = orc.select_boxes(boxes, W, H, k, CROP)
    cx0, cx1 = np.maximum(boxes[:, 0], 0), np.minimum(boxes[:, 2], W)
    cy0, cy1 = np.maximum(boxes[:, 1], 0), np.minimum(boxes[:, 3], H)
    cand = (boxes[:, 4] & 1).astype(bool) & (cx0 < cx1) & (cy0 < cy1)
    u = (cx0 + cx1 - 1) / 2
    frontal = cand & (u >= 333) & (u < 667)
    side = cand & ~frontal
    kept = (out[:, 4] & 1).astype(bool) & cand
    assert kept.sum() == min(k, cand.sum())
    assert (out[~cand] == boxes[~cand]).all() and (rank[~cand] == -1).all()
    if (kept & side).any():
        assert kept[frontal].all()
    for cls in (frontal, side):
        if (kept & cls).any() and (~kept & cls).any():
            assert cy1[kept & cls].min() >= cy1[~kept & cls].max()


def test_crop_edge_uses_the_pixel_centre(orc):
    """The crop is [333, 667) in x for W = 1000: a box over columns 599..733 has centre
    666.0 (in), one over 600..733 has centre 666.5 (in), one over 601..733 has 667.0
    (out)."""
    boxes = np.array([[599, 0, 734, 50, 1], [600, 0, 734, 40, 1], [601, 0, 734, 30, 1],
                      [0, 0, 10, 590, 1]], np.int32)
    _, rank = orc.select_boxes(boxes, W, H, 1, CROP)
    # frontal ones first by bottom: box 0 (50), box 1 (40); then side: box 3 (590), box 2 (30)
    assert rank.tolist() == [0, 1, 3, 2]
