"""Autotuner of the matching launches: kernel variant per path shape, blocks per wave
grid size and whether both levels share one launch, measured on the caller's own
workload and kept in a JSON table.

The register-blocked matching kernel comes in variants (rows of a block per wave,
candidates per lane) that all compute the same costs; blocks per wave and the grid size
only change how work items are dealt, and a shared launch only how they are launched.
None of them changes a result, so the tuner times
each choice on a real workload, requires its output to equal the default's bit for bit,
and keeps the fastest. A table is tied to the device architecture it was measured on.

    table = autotune.tune(run, params)        # run(): one call of the workload
    autotune.save(table, "tune.json")
    autotune.apply(autotune.load("tune.json"))
"""
from __future__ import annotations

import json
from dataclasses import dataclass, field

from . import ocsr

BLOCKS_PER_WAVE = (1, 2, 4)
MATCH_WGS_PER_CU = (4, 8, 16, 32)
DEFAULT_BLOCKS_PER_WAVE = 1
DEFAULT_MATCH_WGS_PER_CU = 16


@dataclass
class Table:
    arch: str
    variants: dict = field(default_factory=dict)   # "bw x bh / nd" -> [rows, cpl, passes]
    blocks_per_wave: int = DEFAULT_BLOCKS_PER_WAVE
    match_wgs_per_cu: int = DEFAULT_MATCH_WGS_PER_CU
    level_launches: int = 0                          # OPTION_LEVEL_LAUNCHES
    timings_ms: dict = field(default_factory=dict)  # choice -> measured time


def shape_key(bw: int, bh: int, nd: int) -> str:
    return f"{bw}x{bh}/{nd}"


def path_shapes(params: dict) -> list[tuple[int, int, int]]:
    """(bw, bh, level candidates) of the far path (level scale 1) and the close path."""
    out = []
    for name, scale in (("far", 1), ("close", params["close_scale"])):
        ph = params[name]
        shape = (ph["bw"], ph["bh"], ocsr.level_candidates(ph, scale))
        if shape not in out:
            out.append(shape)
    return out


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def _time_ms(run, reps: int, warmup: int, trials: int = 3) -> float:
    """Milliseconds per call of `run` submitted back to back (the throughput a caller that
    keeps the stream busy sees): the median over `trials` runs of `reps` calls."""
    import torch
    for _ in range(warmup):
        run()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(trials):
        a.record()
        for _ in range(reps):
            run()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) / reps)
    times.sort()
    return times[len(times) // 2]


def _snapshot(result):
    return result.detach().cpu().clone()


def apply(table: Table, device: int | None = None) -> None:
    """Installs a table's choices in the device's library context."""
    if table.arch != _arch():
        raise ValueError(f"table measured on {table.arch}, device is {_arch()}")
    for key, (rows, cpl, passes) in table.variants.items():
        bw_bh, nd = key.split("/")
        bw, bh = (int(v) for v in bw_bh.split("x"))
        ocsr.set_variant(bw, bh, int(nd), rows, cpl, passes, device)
    ocsr.set_option(ocsr.OPTION_BLOCKS_PER_WAVE, table.blocks_per_wave, device)
    ocsr.set_option(ocsr.OPTION_MATCH_WGS_PER_CU, table.match_wgs_per_cu, device)
    ocsr.set_option(ocsr.OPTION_LEVEL_LAUNCHES, table.level_launches, device)


def reset(params: dict, device: int | None = None) -> None:
    """Restores the library defaults for the paths of `params`."""
    for bw, bh, nd in path_shapes(params):
        ocsr.set_variant(bw, bh, nd, 0, 0, 0, device)
    ocsr.set_option(ocsr.OPTION_BLOCKS_PER_WAVE, DEFAULT_BLOCKS_PER_WAVE, device)
    ocsr.set_option(ocsr.OPTION_MATCH_WGS_PER_CU, DEFAULT_MATCH_WGS_PER_CU, device)
    ocsr.set_option(ocsr.OPTION_LEVEL_LAUNCHES, 0, device)


def tune(run, params: dict, reps: int = 20, warmup: int = 3,
         blocks_per_wave=BLOCKS_PER_WAVE, match_wgs_per_cu=MATCH_WGS_PER_CU,
         device: int | None = None, rounds: int = 2, margin: float = 0.01) -> Table:
    """Tunes the matching launches for the workload `run` (a callable that submits one
    call and returns its result tensor) with parameters `params`.

    Coordinate descent: the variant of each path shape in turn (the others at their
    current best), then blocks per wave, then the grid, then one or two matching
    launches; `rounds` passes over all of them, each starting from the last's choices.
    Each coordinate keeps its current setting (the library default in the first round)
    unless another is faster by more than `margin` (a fraction of its time), so that
    timing noise does not move it. Every choice's output must equal the default
    configuration's exactly; a choice that differs raises, since it would be a library
    defect. The chosen configuration is left installed."""
    reset(params, device)
    ref = _snapshot(run())
    table = Table(arch=_arch())

    def measure(label):
        out = _snapshot(run())
        if not bool((out == ref).all()):
            raise RuntimeError(f"tuning choice {label} changed the results")
        ms = _time_ms(run, reps, warmup)
        table.timings_ms[label] = round(ms, 5)
        return ms

    def pick(current, candidates, apply, label):
        """The fastest of `candidates`, measured after `current`; another replaces
        `current` only when faster by more than the margin. Leaves the pick applied."""
        apply(current)
        best_ms, best = measure(label(current)), current
        for c in candidates:
            if c == current:
                continue
            apply(c)
            ms = measure(label(c))
            if ms < best_ms * (1.0 - margin):
                best_ms, best = ms, c
        apply(best)
        return best

    bpw_now, wgs_now, mode_now = DEFAULT_BLOCKS_PER_WAVE, DEFAULT_MATCH_WGS_PER_CU, 0
    for rnd in range(rounds):
        for bw, bh, nd in path_shapes(params):
            cands = [tuple(v) for v in ocsr.variant_candidates(bw, bh, nd)]
            if not cands:
                continue
            key = shape_key(bw, bh, nd)
            # the library's default for the shape is the first candidate
            now = tuple(table.variants.get(key, cands[0]))
            best = pick(now, cands, lambda v: ocsr.set_variant(bw, bh, nd, *v, device),
                        lambda v: f"round {rnd} variant {key} rows={v[0]} cpl={v[1]} passes={v[2]}")
            table.variants[key] = list(best)

        bpw_now = pick(bpw_now, list(blocks_per_wave),
                       lambda v: ocsr.set_option(ocsr.OPTION_BLOCKS_PER_WAVE, v, device),
                       lambda v: f"round {rnd} blocks_per_wave={v}")
        table.blocks_per_wave = bpw_now

        wgs_now = pick(wgs_now, list(match_wgs_per_cu),
                       lambda v: ocsr.set_option(ocsr.OPTION_MATCH_WGS_PER_CU, v, device),
                       lambda v: f"round {rnd} match_wgs_per_cu={v}")
        table.match_wgs_per_cu = wgs_now

        mode_now = pick(mode_now, [0, 1, 2],
                        lambda v: ocsr.set_option(ocsr.OPTION_LEVEL_LAUNCHES, v, device),
                        lambda v: f"round {rnd} level_launches={v}")
        table.level_launches = mode_now
    return table


def to_json(table: Table) -> str:
    return json.dumps({"arch": table.arch, "variants": table.variants,
                       "blocks_per_wave": table.blocks_per_wave,
                       "match_wgs_per_cu": table.match_wgs_per_cu,
                       "level_launches": table.level_launches,
                       "timings_ms": table.timings_ms}, indent=1, sort_keys=True)


def from_json(text: str) -> Table:
    d = json.loads(text)
    t = Table(arch=d["arch"], variants={k: [int(x) for x in v] for k, v in d["variants"].items()},
              blocks_per_wave=int(d["blocks_per_wave"]),
              match_wgs_per_cu=int(d["match_wgs_per_cu"]),
              level_launches=int(d.get("level_launches", 0)),
              timings_ms=dict(d.get("timings_ms", {})))
    for key, v in t.variants.items():
        bw_bh, nd = key.split("/")
        bw, bh = (int(x) for x in bw_bh.split("x"))
        if len(v) != 3 or tuple(v) not in ocsr.variant_candidates(bw, bh, int(nd)):
            raise ValueError(f"table entry {key}: no kernel {v} (rows, cpl, passes) covers it")
    if not 1 <= t.blocks_per_wave <= 8 or not 1 <= t.match_wgs_per_cu <= 64 or t.level_launches not in (0, 1, 2):
        raise ValueError("table launch settings out of range")
    return t


def save(table: Table, path: str) -> None:
    with open(path, "w") as f:
        f.write(to_json(table))


def load(path: str) -> Table:
    with open(path) as f:
        return from_json(f.read())
