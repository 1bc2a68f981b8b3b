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
    "aggregate": ["paper_2604_07980_amd/csrc/match.hip", "paper_2604_07980_amd/csrc/dev_match.hpp",
                  "paper_2604_07980_amd/csrc/dev_common.hpp",
                  "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
    "dense": ["paper_2604_07980_amd/csrc/dense.hip", "paper_2604_07980_amd/csrc/ocsr_internal.hpp"],
}

# rocprofv3 kernel names (demangled) of each reported kernel
KERNEL_PATTERNS = {
    "census": r"frame_census_kernel",
    "match": r"match_pair_kernel|match_tiled_kernel",
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


def _counter_means(run_dir: str, counter: str, pattern: str) -> tuple[float, int]:
    """Mean per dispatch (KiB as reported) of `counter` over the dispatches whose
    kernel name matches `pattern`."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    per_dispatch: dict[str, float] = {}
    for fn in files:
        for r in csv.DictReader(open(fn)):
            if r.get("Counter_Name") != counter or not re.search(pattern, r.get("Kernel_Name", "")):
                continue
            key = fn + ":" + r.get("Dispatch_Id", r.get("Correlation_Id", ""))
            per_dispatch[key] = per_dispatch.get(key, 0.0) + float(r["Counter_Value"])
    if not per_dispatch:
        raise ValueError(f"no {counter} records for kernels matching {pattern!r} in {run_dir}")
    vals = list(per_dispatch.values())
    return sum(vals) / len(vals), len(vals)


def traffic_entry(kernel: str, fetch_dir: str, write_dir: str, copy_fetch_dir: str,
                  copy_write_dir: str, copy_bytes: int, command: str) -> dict:
    pat = KERNEL_PATTERNS[kernel]
    f_k, nf = _counter_means(fetch_dir, "FETCH_SIZE", pat)
    w_k, nw = _counter_means(write_dir, "WRITE_SIZE", pat)
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
    b = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        b.add_argument("--" + k.replace("_", "-"), required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--kernel", required=True, choices=sorted(KERNEL_SOURCES))
    b.add_argument("--workload", required=True, help="workload name the entry is filed under")
    b.add_argument("--command", required=True)
    b.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        sys.stdout.write(stats_markdown(args.csv, args.command))
        return
    entry = traffic_entry(args.kernel, args.fetch, args.write, args.copy_fetch, args.copy_write,
                          args.copy_bytes, args.command)
    table = json.load(open(args.out)) if os.path.exists(args.out) else {}
    table.setdefault(args.workload, {})[args.kernel] = entry
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps(entry, indent=1))


if __name__ == "__main__":
    main()
