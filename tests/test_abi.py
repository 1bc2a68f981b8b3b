"""Host-side checks of the C ABI: the built library loads and exports every function
that include/*.h declares, and the binding's structures match the header's sizes.
No GPU and no compute calls."""
import ctypes as C
import glob
import os
import re

import pytest

from paper_2604_07980_amd import ocsr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(ocsr_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(ocsr.LIB_PATH):
        from paper_2604_07980_amd import build
        build.build()
    return ocsr.load()


def test_exports_every_declared_symbol(built):
    declared = _declared_functions()
    assert declared, "no declarations found"
    missing = [n for n in sorted(declared) if not hasattr(built, n)]
    assert not missing, missing
    assert set(ocsr.EXPORTS) == declared


def test_abi_version_and_host_only_calls(built):
    assert built.ocsr_abi_version() == 3
    assert built.ocsr_last_error() == b""
    # workspace sizing is pure host arithmetic
    a = built.ocsr_match_workspace_bytes(32, 1 << 16)
    b = built.ocsr_match_workspace_bytes(64, 1 << 16)
    assert 0 < a < b
    fp = ocsr.FrameParams(3, 4, 1, 2)
    f = built.ocsr_frame_workspace_bytes(1920, 1080, C.byref(fp), 32, 1 << 16)
    assert f >= a + 2 * 1920 * 1080 * 8 + 2 * 960 * 540 * 8
    assert built.ocsr_frame_workspace_bytes(0, 1080, C.byref(fp), 32, 1 << 16) == 0


def test_rect_workspace_sizing(built):
    """Host arithmetic: three int16 maps per offset plus the partial counts, each block
    256-byte aligned; 0 for an invalid description."""
    rp = ocsr.RectParams(0, 10, 100, 20, -2, 2, 0, 31, 2, 1, 0)
    maps = 3 * 5 * 100 * 20 * 2
    parts = 5 * 20 * 1 * 4
    a256 = lambda v: (v + 255) // 256 * 256
    assert built.ocsr_rect_workspace_bytes(C.byref(rp)) == a256(maps) + a256(parts)
    for bad in (dict(roi_w=0), dict(delta_min=3), dict(delta_min=-40, delta_max=40)):
        q = ocsr.RectParams(0, 10, 100, 20, -2, 2, 0, 31, 2, 1, 0)
        for k, v in bad.items():
            setattr(q, k, v)
        assert built.ocsr_rect_workspace_bytes(C.byref(q)) == 0


def test_struct_sizes_match_header():
    assert C.sizeof(ocsr.MatchParams) == 4 + 4 + 2 * 24 + 3 * 4 + 4 + 2 * 4 + 3 * 4 + 2 * 4
    assert C.sizeof(ocsr.Level) == 2 * 8 + 6 * 4
    assert C.sizeof(ocsr.CensusJob) == 2 * 8 + 6 * 4
    assert C.sizeof(ocsr.Debug) == 2 * 4 + 4 * 8
    assert ocsr.BLOCK_RECORD_DTYPE.itemsize == 80
    assert C.sizeof(ocsr.SelectParams) == 5 * 4
    assert C.sizeof(ocsr.RectParams) == 11 * 4


def test_header_constants_match_binding():
    src = open(os.path.join(ROOT, "include", "ocsr.h")).read()
    def const(name):
        return int(re.search(rf"#define {name} \(?(-?\d+)", src).group(1))
    assert const("OCSR_MAX_CANDIDATES") == ocsr.MAX_CANDIDATES
    assert const("OCSR_MAX_DY") == ocsr.MAX_DY
    assert const("OCSR_MAX_DY_CANDIDATES") == ocsr.MAX_DY_CANDIDATES
    assert const("OCSR_MAX_SELECT_BOXES") == ocsr.MAX_SELECT_BOXES
    assert const("OCSR_MAX_RECT_OFFSETS") == ocsr.MAX_RECT_OFFSETS
    assert const("OCSR_MAX_CENSUS_JOBS") == ocsr.MAX_CENSUS_JOBS
    for k, name in enumerate(ocsr.REASONS):
        assert const(f"OCSR_REASON_{name}") == k


def test_vertical_limits_stated_in_the_header():
    """The header's vertical-range limits for 8 x 8 paths, restated from the per-wave LDS
    rule: a 1/4 workgroup share of 64 KB holds the strip rows (all ROWS + ndy - 1 when they
    fit 16 loads per lane, else a ring of ROWS + 1), the template and two uint16 cost
    tables; and nd * ndy <= OCSR_MAX_DY_CANDIDATES."""
    def r16(v):
        return (v + 15) // 16 * 16

    def strip(rows, nd):
        return -(-nd // 32) * 32 + rows - 1

    def lds(rows, nd, ndy):
        full = (rows + ndy - 1) * strip(rows, nd) <= 64 * 16
        lr = rows + ndy - 1 if full else rows + 1
        return r16(8 * lr * strip(rows, nd)) + r16(8 * rows * rows) + 2 * r16(2 * nd * ndy)

    def most(nd):
        return max(n for n in range(1, 200) if nd * n <= ocsr.MAX_DY_CANDIDATES and 4 * lds(8, nd, n) <= 65536)
    assert most(96) == 21 and most(128) == 12
    assert strip(8, 160) <= 3 * 64 < strip(8, 161)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N > 1 exits with a message before touching a GPU."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""
