"""The no-allocation matching entry point (ocsr_match_boxes_noalloc) against
ocsr_match_boxes on the same descriptors: results identical bit for bit on two calls in
a row, the second with a smaller input (the shared scratch keeps the first call's
contents), and sizes beyond the scratch rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2604_07980_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _levels(lib, sc, p):
    L, R = _cuda(sc.left), _cuda(sc.right)
    s = p["close_scale"]
    return lib.census_many([L, R, L, R], [1, 1, s, s], p["sx"], p["sy"], p["sentinel"])


def _same(a, b):
    return torch.equal(a, b)


def test_noalloc_equals_match_boxes_on_two_calls(lib):
    big = synth.scene_realistic()
    p_big = synth.params_for(2)
    small = synth.scene_tiny()
    p_small = synth.params_for(1)
    c_big, c_small = _levels(lib, big, p_big), _levels(lib, small, p_small)
    b_big, b_small = _cuda(big.boxes), _cuda(small.boxes)
    print("noalloc: realistic 1080p frame, 64 boxes; then 640x480, 4 boxes", flush=True)
    for (c, b, p, cap) in ((c_big, b_big, p_big, 1 << 16), (c_small, b_small, p_small, 1 << 12)):
        want = lib.match_boxes(*c, b, p, cap_blocks=cap)
        got = lib.match_boxes_noalloc(*c, b, p, cap_blocks=cap)
        torch.cuda.synchronize()
        assert _same(got, want), (lib.results_to_numpy(got), lib.results_to_numpy(want))
        r = lib.results_to_numpy(got)
        assert (r["valid"] == 1).sum() >= 3
    # the first input again after the smaller one
    again = lib.match_boxes_noalloc(*c_big, b_big, p_big, cap_blocks=1 << 16)
    assert _same(again, lib.match_boxes(*c_big, b_big, p_big, cap_blocks=1 << 16))


def test_noalloc_rejects_sizes_beyond_scratch(lib):
    sc = synth.scene_tiny()
    p = synth.params_for(1)
    c = _levels(lib, sc, p)
    b = _cuda(sc.boxes)
    with pytest.raises(lib.OcsrError) as e:
        lib.match_boxes_noalloc(*c, b, p, cap_blocks=1 << 22)
    assert e.value.code == lib.E_CAPACITY
    assert "scratch" in str(e.value)
