"""The library's host-side offset filter (ocsr_rect_filter_*, Sec. 5.1 filter equations)
against the oracle's, over random count sequences; and its argument checks. Host code
only: no GPU is needed."""
import os

import numpy as np
import pytest

from paper_2604_07980_amd import ocsr


@pytest.fixture(scope="module")
def host():
    if not os.path.exists(ocsr.LIB_PATH):
        from paper_2604_07980_amd import build
        build.build()
    ocsr.load()
    return ocsr


@pytest.mark.parametrize("window,max_step,initial", [(1, 0, 0), (1, 100, 0), (3, 1, 0), (5, 2, -3),
                                                     (8, 1, 2), (15, 4, 0)])
def test_filter_equals_oracle(host, orc, window, max_step, initial):
    rng = np.random.default_rng(window * 31 + max_step)
    n, lo, T = 9, -4, 200
    # counts with a drifting true offset, noise and frequent ties
    truth = np.cumsum(rng.integers(-1, 2, T)).clip(-4, 4)
    counts = rng.integers(0, 50, (T, n))
    counts[np.arange(T), truth - lo] += rng.integers(0, 60, T)
    counts[rng.random((T, n)) < 0.1] = counts.max()   # ties with the top
    raw_o, filt_o = orc.rect_filter(counts, lo, window, max_step, initial)
    f = host.RectFilter(window, max_step, initial)
    got = [f.update(c, lo) for c in counts]
    assert [g[0] for g in got] == raw_o.tolist()
    assert [g[1] for g in got] == filt_o.tolist()


def test_filter_rejects_bad_arguments(host):
    for args in ((0, 1, 0), (1, -1, 0), (2000, 1, 0)):
        with pytest.raises(host.OcsrError) as e:
            host.RectFilter(*args)
        assert e.value.code == host.E_INVALID
    f = host.RectFilter(3, 1)
    with pytest.raises(host.OcsrError):
        f.update(np.zeros(0, np.int32), 0)
    with pytest.raises(host.OcsrError):
        f.update(np.zeros(host.MAX_RECT_OFFSETS + 1, np.int32), 0)
