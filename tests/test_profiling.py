"""Host-side checks of the rocprofv3 summaries (paper_2604_07980_amd/profiling.py) on small
hand-made CSV files: the last-N dispatch window, the copy-calibrated traffic scaling, the
SQ-counter table and the source hashes."""
import csv
import os

import pytest

from paper_2604_07980_amd import profiling

CLOSE = "void ocsr::(anonymous namespace)::match_level_kernel<ocsr::dev::HalfMatcher<3>, 4>(ocsr::MatchParamsDev)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _counters(run_dir, counter, per_dispatch):
    """counter_collection.csv with each dispatch's value split over two rows (two XCDs)."""
    os.makedirs(run_dir, exist_ok=True)
    rows = []
    for did, (name, value) in enumerate(per_dispatch, start=1):
        for half in (0.25, 0.75):
            rows.append({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": counter,
                         "Counter_Value": value * half})
    _write(os.path.join(run_dir, "run_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_trace_window_keeps_the_last_dispatches(tmp_path):
    path = tmp_path / "run_kernel_trace.csv"
    # three set-up dispatches of 50 us, then five timed ones of 10 us
    rows = [{"Kernel_Name": CLOSE, "Start_Timestamp": 1000 * i, "End_Timestamp": 1000 * i + d}
            for i, d in enumerate([50000] * 3 + [10000] * 5)]
    _write(path, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    md = profiling.trace_markdown(str(path), last=5)
    line = next(l for l in md.splitlines() if "HalfMatcher" in l)
    cells = [c.strip() for c in line.split("|")]
    assert cells[2] == "5" and cells[3] == "10.00" and cells[5] == "10.00"
    md_all = profiling.trace_markdown(str(path), last=100)
    line = next(l for l in md_all.splitlines() if "HalfMatcher" in l)
    assert [c.strip() for c in line.split("|")][3] == f"{(3 * 50 + 5 * 10) / 8:.2f}"


def test_traffic_scaled_by_the_copy_and_windowed(tmp_path):
    copy_bytes = 1 << 20
    _counters(tmp_path / "cf", "FETCH_SIZE", [(COPY, 512.0)])      # 2 KiB per unit
    _counters(tmp_path / "cw", "WRITE_SIZE", [(COPY, 1024.0)])     # 1 KiB per unit
    # a set-up dispatch with a different count, then the timed ones
    _counters(tmp_path / "kf", "FETCH_SIZE", [(CLOSE, 9999.0), (CLOSE, 100.0), (CLOSE, 300.0)])
    _counters(tmp_path / "kw", "WRITE_SIZE", [(CLOSE, 7.0), (CLOSE, 2.0), (CLOSE, 4.0)])
    e = profiling.traffic_entry("match_close", str(tmp_path / "kf"), str(tmp_path / "kw"),
                                str(tmp_path / "cf"), str(tmp_path / "cw"), copy_bytes, "cmd", last=2)
    assert e["dispatches"] == [2, 2]
    assert e["fetch_scale"] == pytest.approx(2048.0) and e["write_scale"] == pytest.approx(1024.0)
    assert e["fetch_bytes"] == pytest.approx(200.0 * 2048.0)
    assert e["write_bytes"] == pytest.approx(3.0 * 1024.0)
    assert e["source_sha256"] == profiling.source_hash("match_close")
    md = profiling.traffic_markdown({"match_close": e})
    assert "match_close" in md and "2048 fetched / 1024 written" in md


def test_sq_table_relative_to_the_chain_kernel(tmp_path):
    rows = []
    did = 0
    # the chain kernel: 4 VALU instructions x 4 cycles on 1024 SIMDs over 16 cycles of
    # 32 shader engines -> raw busy 1.0
    for name, valu, busy in (("int_rate_kernel", 4096.0, 512.0), (CLOSE, 2048.0, 512.0)):
        did += 1
        for c, v in (("SQ_INSTS_VALU", valu), ("SQ_BUSY_CYCLES", busy), ("SQ_WAVES", 64.0),
                     ("SQ_WAVE_CYCLES", 100.0), ("SQ_WAIT_INST_ANY", 25.0), ("SQ_INSTS_SALU", 1.0),
                     ("SQ_INSTS_LDS", 2.0), ("SQ_INSTS_VMEM_RD", 3.0)):
            rows.append({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v})
    path = tmp_path / "run_counter_collection.csv"
    _write(path, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    md = profiling.sq_markdown(str(path), last=10)
    close = next(l for l in md.splitlines() if "HalfMatcher" in l)
    cells = [c.strip() for c in close.split("|")]
    assert cells[-2] == "0.50"          # half the chain kernel's VALU rate
    assert cells[-3] == "0.25"          # wait / wave cycles
    assert cells[8] == "32"             # VALU instructions per wave


def test_source_hash_covers_every_reported_kernel():
    for k in profiling.KERNEL_SOURCES:
        assert len(profiling.source_hash(k)) == 64
    assert profiling.source_hash("match_close") == profiling.source_hash("match_far")
