"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_2604_07980_amd.profiling stats <kernel_stats.csv> --command "..."
    python -m paper_2604_07980_amd.profiling traffic --fetch <dir> --write <dir> \\
        --copy-fetch <dir> --copy-write <dir> --copy-bytes N --kernel census \\
        --workload batch_16x1920x1200 --command "..."

`stats` turns a `--kernel-trace --stats` kernel table into a short markdown table.
`traffic` turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of a workload, plus the
same two counters read for a plain device copy of known size, into HBM bytes per launch
of one kernel: each counter's per-dispatch mean is scaled by the bytes the copy really
moves over what the counter reported for it. Entries are filed by workload, then kernel;
each records a hash of the kernel's source files, so a reader can tell whether the
kernel changed since.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# source files each reported kernel is built from (relative to the repository root)
KERNEL_SOURCES = {
    "census": ["paper_2604_07980_amd/csrc/dev_census.hpp", "paper_2604_07980_amd/csrc/match.hip",
               "paper_2604_07980_amd/csrc/dev_match.hpp", "paper_2604_07980_amd/csrc/dev_common.hpp",
               "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
    "match": ["paper_2604_07980_amd/csrc/match.hip", "paper_2604_07980_amd/csrc/dev_match.hpp",
              "paper_2604_07980_amd/csrc/dev_common.hpp", "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
    "match_close": ["paper_2604_07980_amd/csrc/match.hip", "paper_2604_07980_amd/csrc/dev_match.hpp",
                    "paper_2604_07980_amd/csrc/dev_common.hpp", "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
    "match_far": ["paper_2604_07980_amd/csrc/match.hip", "paper_2604_07980_amd/csrc/dev_match.hpp",
                  "paper_2604_07980_amd/csrc/dev_common.hpp", "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
    "plan": ["paper_2604_07980_amd/csrc/match.hip", "paper_2604_07980_amd/csrc/dev_match.hpp",
             "paper_2604_07980_amd/csrc/dev_census.hpp", "paper_2604_07980_amd/csrc/dev_common.hpp",
             "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
    "aggregate": ["paper_2604_07980_amd/csrc/match.hip", "paper_2604_07980_amd/csrc/dev_match.hpp",
                  "paper_2604_07980_amd/csrc/dev_common.hpp",
                  "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
    "dense": ["paper_2604_07980_amd/csrc/dense.hip", "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
}

# rocprofv3 kernel names (demangled) of each reported kernel
KERNEL_PATTERNS = {
    "census": r"frame_census_kernel|census_list_kernel",
    "plan": r"plan_tiles_kernel",
    "match": r"match_pair_kernel|match_tiled_kernel|match_pair2_kernel|match_level_kernel",
    # the batch workload's tuned variants: the row-half matcher serves the close level,
    # the generic or four-block matcher the far level
    "match_close": r"match_level_kernel<ocsr::dev::HalfMatcher",
    "match_far": r"match_level_kernel<ocsr::dev::(GenericMatcher|QuadMatcher)",
    "aggregate": r"aggregate_kernel",
    "dense": r"dense_kernel",
    "copy": r"copyBuffer",
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    name = name.replace("ocsr::(anonymous namespace)::", "")
    name = re.sub(r"\(.*", "", name)
    return name.replace("void ", "").strip()


def stats_markdown(path: str, command: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"Command: `{command}`", "",
           "| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share |",
           "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.1f}% |")
    return "\n".join(out) + "\n"


def trace_markdown(path: str, last: int, top: int = 12) -> str:
    """Per-kernel durations over the last `last` dispatches of each kernel in a
    `--kernel-trace` CSV (the timed region of a command whose set-up launches the same
    kernels first)."""
    per: dict[str, list[tuple[int, float]]] = {}
    for r in csv.DictReader(open(path)):
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        per.setdefault(r["Kernel_Name"], []).append((t0, (t1 - t0) / 1e3))
    rows = []
    for name, v in per.items():
        v.sort()
        d = [x[1] for x in v[-last:]]
        rows.append((sum(d), name, d))
    rows.sort(key=lambda r: -r[0])
    total = sum(r[0] for r in rows)
    out = [f"Last {last} dispatches of each kernel, from the kernel trace:", "",
           "| Kernel | Dispatches | Average (us) | Min (us) | Max (us) | Share |",
           "|---|---|---|---|---|---|"]
    for tot, name, d in rows[:top]:
        out.append(f"| `{_short(name)}` | {len(d)} | {tot / len(d):.2f} | {min(d):.2f} | "
                   f"{max(d):.2f} | {100 * tot / total:.1f}% |")
    return "\n".join(out) + "\n"


SQ_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_WAVES",
               "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY")


def sq_markdown(path: str, last: int, ref: str = "int_rate_kernel", n_se: int = 32,
                n_simd: int = 1024) -> str:
    """Instruction counters per dispatch (the last `last` dispatches of each kernel) of one
    `--pmc` run of the SQ_ counters. VALU busy is INSTS_VALU x 4 cycles over SIMDs x
    kernel cycles (BUSY_CYCLES summed over the shader engines / their number), divided by
    the same figure for `ref`, the chain kernel that runs the VALU at the measured peak."""
    per: dict[tuple[str, int], dict[str, float]] = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] not in SQ_COUNTERS:
            continue
        d = per.setdefault((r["Kernel_Name"], int(r["Dispatch_Id"])), {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    by: dict[str, list[dict[str, float]]] = {}
    for (name, _), d in sorted(per.items(), key=lambda kv: kv[0][1]):
        by.setdefault(name, []).append(d)

    def mean(v):
        v = v[-last:]
        return {c: sum(x.get(c, 0.0) for x in v) / len(v) for c in SQ_COUNTERS}, len(v)

    def raw_busy(m):
        cyc = m["SQ_BUSY_CYCLES"] / n_se
        return 4 * m["SQ_INSTS_VALU"] / (n_simd * cyc) if cyc else 0.0

    ref_busy = next((raw_busy(mean(v)[0]) for n, v in by.items() if ref in n), 0.0) or 1.0
    out = [f"Means over the last {last} dispatches of each kernel; VALU busy relative to "
           f"`{ref}` (raw figure {ref_busy:.3f}).", "",
           "| Kernel | Dispatches | VALU instr | SALU instr | LDS instr | VMEM rd instr | Waves | "
           "VALU instr / wave | Wait / wave cycles | VALU busy |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    rows = [(n, *mean(v)) for n, v in by.items()]
    rows.sort(key=lambda r: -r[1]["SQ_BUSY_CYCLES"])
    for n, m, k in rows:
        if _short(n).startswith("at::") or "rocclr" in n:
            continue
        w = max(1.0, m["SQ_WAVES"])
        out.append(f"| `{_short(n)}` | {k} | {m['SQ_INSTS_VALU']:.4g} | {m['SQ_INSTS_SALU']:.4g} | "
                   f"{m['SQ_INSTS_LDS']:.4g} | {m['SQ_INSTS_VMEM_RD']:.4g} | {m['SQ_WAVES']:.0f} | "
                   f"{m['SQ_INSTS_VALU'] / w:.0f} | "
                   f"{m['SQ_WAIT_INST_ANY'] / max(1.0, m['SQ_WAVE_CYCLES']):.2f} | "
                   f"{raw_busy(m) / ref_busy:.2f} |")
    return "\n".join(out) + "\n"


def _counter_means(run_dir: str, counter: str, pattern: str, last: int = 0) -> tuple[float, int]:
    """Mean per dispatch (KiB as reported) of `counter` over the dispatches whose
    kernel name matches `pattern` (the last `last` of them when last > 0)."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    per_dispatch: dict[str, float] = {}
    for fn in files:
        for r in csv.DictReader(open(fn)):
            if r.get("Counter_Name") != counter or not re.search(pattern, r.get("Kernel_Name", "")):
                continue
            key = (fn, int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0))
            per_dispatch[key] = per_dispatch.get(key, 0.0) + float(r["Counter_Value"])
    if not per_dispatch:
        raise ValueError(f"no {counter} records for kernels matching {pattern!r} in {run_dir}")
    vals = [per_dispatch[k] for k in sorted(per_dispatch)]
    if last > 0:
        vals = vals[-last:]
    return sum(vals) / len(vals), len(vals)


def traffic_entry(kernel: str, fetch_dir: str, write_dir: str, copy_fetch_dir: str,
                  copy_write_dir: str, copy_bytes: int, command: str, last: int = 0) -> dict:
    pat = KERNEL_PATTERNS[kernel]
    f_k, nf = _counter_means(fetch_dir, "FETCH_SIZE", pat, last)
    w_k, nw = _counter_means(write_dir, "WRITE_SIZE", pat, last)
    f_c, _ = _counter_means(copy_fetch_dir, "FETCH_SIZE", KERNEL_PATTERNS["copy"])
    w_c, _ = _counter_means(copy_write_dir, "WRITE_SIZE", KERNEL_PATTERNS["copy"])
    f_scale, w_scale = copy_bytes / f_c, copy_bytes / w_c
    return {"kernel": kernel, "source_sha256": source_hash(kernel),
            "fetch_bytes": f_k * f_scale, "write_bytes": w_k * w_scale,
            "fetch_counter_mean": f_k, "write_counter_mean": w_k, "dispatches": [nf, nw],
            "copy_bytes": copy_bytes, "copy_fetch_counter": f_c, "copy_write_counter": w_c,
            "fetch_scale": f_scale, "write_scale": w_scale, "command": command}


def traffic_markdown(table: dict) -> str:
    out = ["| Kernel | Dispatches | FETCH_SIZE mean | WRITE_SIZE mean | Fetch (MB) | Write (MB) |",
           "|---|---|---|---|---|---|"]
    for k, e in sorted(table.items()):
        out.append(f"| {k} | {e['dispatches'][0]} | {e['fetch_counter_mean']:.1f} | "
                   f"{e['write_counter_mean']:.1f} | {e['fetch_bytes'] / 1e6:.3f} | "
                   f"{e['write_bytes'] / 1e6:.3f} |")
    e = next(iter(table.values()))
    out += ["", f"Copy reference: {e['copy_bytes']} bytes read and written per dispatch; "
                f"FETCH_SIZE read {e['copy_fetch_counter']:.1f} and WRITE_SIZE "
                f"{e['copy_write_counter']:.1f} for it, so one counter unit is "
                f"{e['fetch_scale']:.0f} fetched / {e['write_scale']:.0f} written bytes."]
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--trace", default="", help="kernel_trace.csv of the same run")
    a.add_argument("--last", type=int, default=0,
                   help="with --trace: also tabulate the last N dispatches of each kernel")
    q = sub.add_parser("sq")
    q.add_argument("csv", help="counter_collection.csv of a --pmc run of the SQ_ counters")
    q.add_argument("--last", type=int, default=60)
    q.add_argument("--command", required=True)
    b = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        b.add_argument("--" + k.replace("_", "-"), required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--kernel", required=True, choices=sorted(KERNEL_SOURCES))
    b.add_argument("--workload", required=True, help="workload name the entry is filed under")
    b.add_argument("--command", required=True)
    b.add_argument("--last", type=int, default=0,
                   help="average over the last N dispatches of the kernel only (the timed region)")
    b.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        sys.stdout.write(stats_markdown(args.csv, args.command))
        if args.trace and args.last > 0:
            sys.stdout.write("\n" + trace_markdown(args.trace, args.last))
        return
    if args.cmd == "sq":
        sys.stdout.write(f"Command: `{args.command}`\n\n" + sq_markdown(args.csv, args.last))
        return
    entry = traffic_entry(args.kernel, args.fetch, args.write, args.copy_fetch, args.copy_write,
                          args.copy_bytes, args.command, args.last)
    table = json.load(open(args.out)) if os.path.exists(args.out) else {}
    table.setdefault(args.workload, {})[args.kernel] = entry
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps(entry, indent=1))


if __name__ == "__main__":
    main()
