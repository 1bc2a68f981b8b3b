#!/usr/bin/env python3
"""Benchmark of the object-centric census template-matching path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload (one step = the whole path over one frame): the realistic 1920x1080 frame --
census of both views at both levels (on the 64x32 tiles the boxes' searches read), then
per-box planning, forward/backward Hamming
block search with WTA and parabola, L/R check, aggregation and depth, for 32 ranged
boxes (19 far, 13 close) plus 32 occluder boxes. Inputs are resident in HBM before
the timed region starts.

Prints one JSON line: Gcost/s (one cost = one 64-bit Hamming term, forward or
backward) over the timed steps, per-frame p50/p99 latency, the dominant kernel's
roofline, and the CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "box-block disparity evals/sec (Gcost/s) + per-frame p50/p99 latency, 1 MI355X"
INT_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12      # int32 VALU lane-ops/s: CUs x lanes x clock
HBM_PEAK_GBS = 8000.0
CENSUS_OPS_PER_CMP = 1                        # one lane-op per informative comparison bit
MATCH_OPS_PER_COST = 4                        # 2 x v_xor_b32 + 2 x v_bcnt_u32_b32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--latency-steps", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=40,
                    help="timed repetitions of the 16-frame batch (0 skips the batch section)")
    ap.add_argument("--serve-requests", type=int, default=600,
                    help="requests of the serving section at 120/s (0 skips it)")
    ap.add_argument("--serve-pool", type=int, default=2,
                    help="pre-rendered image pairs per serving resolution")
    ap.add_argument("--vertical-steps", type=int, default=100,
                    help="frames of the vertical-range workload (0: skip)")
    ap.add_argument("--rect-steps", type=int, default=50,
                    help="frames of the rectification-offset workload (0: skip)")
    ap.add_argument("--dense-steps", type=int, default=20,
                    help="timed repetitions of the dense counterpart (0 skips it)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device-to-device copy of MB megabytes five times "
                         "(the reference kernel that scales the HBM byte counters)")
    ap.add_argument("--fused", action="store_true",
                    help="run the one-launch persistent kernel instead of the multi-launch path")
    return ap.parse_args()


def cpu_baseline(sc, params, costs_per_frame, seconds):
    """The oracle as it stands, on the host cores, repeated on the same frame."""
    from oracle import oracle as orc
    if not os.path.exists(orc.LIB):
        orc.build()
    cores = len(os.sched_getaffinity(0))
    reps = 0
    t0 = time.perf_counter()
    while True:
        orc.run_scene(sc.left, sc.right, params, sc.boxes, threads=cores)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": costs_per_frame * reps / el / 1e9, "unit": "Gcost/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{reps} repetitions of the realistic 1920x1080 frame (census of both views "
                      f"at both levels + matching of 64 boxes), {el:.1f} s, OpenMP over rows/boxes",
            "ms_per_frame": 1e3 * el / reps}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter measurement
    (profiles/traffic.json), or None when there is none or the kernel's sources changed
    since it was taken."""
    from paper_2604_07980_amd import profiling
    key = {"census": "census", "match": "match", "match_close": "match",
           "match_far": "match", "aggregate": "aggregate"}.get(kernel)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    if key is None or not os.path.exists(path):
        return None
    entry = json.load(open(path)).get(key)
    if not entry or entry.get("source_sha256") != profiling.source_hash(key):
        return None
    return round(entry["fetch_bytes"] + entry["write_bytes"])


def frame_costs(ocsr, L, R, boxes, p):
    """Costs, block evaluations and blocks of one frame, from the library's block records."""
    import numpy as np
    g = ocsr.census_many([L, R, L, R], [1, 1, p["close_scale"], p["close_scale"]])
    _, extra = ocsr.match_boxes(*g, boxes, p, debug=True, cap_blocks=1 << 16)
    nb, rec, _, _ = ocsr.debug_to_numpy(extra)
    el = rec["eligible"] == 1
    pts = np.array([bin(int(m)).count("1") for m in rec["mask"]], dtype=np.int64)
    far = rec["level_scale"] == 1
    # vertical offsets per block: floor(dy_min / s) .. ceil(dy_max / s) on its level
    s = rec["level_scale"].astype(np.int64)
    ndy = -(-p.get("dy_max", 0) // s) - p.get("dy_min", 0) // s + 1
    cand = rec["nd"] * ndy
    return {"costs": int((pts * cand * el).sum()) * 2,
            "costs_far": int((pts * cand * (el & far)).sum()) * 2,
            "evals": int((cand * el).sum()) * 2,
            "blocks": int(nb)}


def vertical_section(ocsr, synth, steps, warmup):
    """The 1080p frame with its right view 2 rows low, searched over dy in [-3, 3] (7
    offsets on the far level, 5 on the close level): whole-frame time and the rate of the
    dy matching kernel (both levels in one launch; the same op count per Hamming cost as
    the horizontal kernels)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    sc = synth.scene_realistic()
    p = dict(synth.params_for(2), dy_min=-3, dy_max=3)
    L = torch.from_numpy(sc.left).to(dev)
    R = torch.from_numpy(synth.drift_rows(sc.right, 2)).to(dev)
    boxes = torch.from_numpy(sc.boxes).to(dev)
    fw = frame_costs(ocsr, L, R, boxes, p)
    ws = ocsr.Workspace()
    out = torch.empty((boxes.shape[0], 8), dtype=torch.int32, device=dev)

    def step():
        ocsr.range_frame(L, R, boxes, p, workspace=ws, out=out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    ocsr.reset_timing()
    ocsr.set_timing(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ocsr.set_timing(False)
    kern = {}
    work = {"match": fw["costs"] * MATCH_OPS_PER_COST}
    for name in ("census", "match", "aggregate"):
        cnt, tot = ocsr.kernel_time(name)
        if cnt:
            kern[name] = {"avg_us": round(1e3 * tot / cnt, 3)}
            if name in work:
                tops = work[name] / (1e-3 * tot / cnt) / 1e12
                kern[name].update(tops=round(tops, 3), frac=round(tops / INT_PEAK_TOPS, 4))
    res = ocsr.results_to_numpy(out)
    return {"workload": "realistic_1080p, right view 2 rows low, dy -3..3 (far 7, close 5 "
                        "level offsets)",
            "ms_per_step": round(ms, 4), "costs_per_frame": fw["costs"],
            "gcost_per_s": round(fw["costs"] / (ms * 1e-3) / 1e9, 3),
            "valid_boxes": int(res["valid"].sum()), "kernels": kern}


def batch_section(ocsr, synth, steps, warmup):
    """16 frames of 1920x1200, min(128, Poisson(40)) boxes each: one batch call against
    16 per-frame calls on the same inputs, with identical outputs required."""
    import torch
    from paper_2604_07980_amd import accounting
    dev = torch.device("cuda:0")
    p = synth.params_for(3)
    scenes = [synth.scene_batch_frame(f) for f in range(16)]
    imgs = [(torch.from_numpy(s.left).to(dev), torch.from_numpy(s.right).to(dev)) for s in scenes]
    fboxes = [torch.from_numpy(s.boxes).to(dev) for s in scenes]
    boxes = torch.cat(fboxes).contiguous()
    frames = [(L, R, b.shape[0]) for (L, R), b in zip(imgs, fboxes)]
    work = [frame_costs(ocsr, L, R, b, p) for (L, R), b in zip(imgs, fboxes)]
    costs = sum(w["costs"] for w in work)
    ws_b, ws_f = ocsr.Workspace(), ocsr.Workspace()
    out_b = torch.empty((boxes.shape[0], 8), dtype=torch.int32, device=dev)
    outs_f = [torch.empty((b.shape[0], 8), dtype=torch.int32, device=dev) for b in fboxes]

    def batch():
        ocsr.range_batch(frames, boxes, p, workspace=ws_b, out=out_b)

    def per_frame():
        for (L, R), b, o in zip(imgs, fboxes, outs_f):
            ocsr.range_frame(L, R, b, p, workspace=ws_f, out=o)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / steps

    ms_default = timed(batch)
    # kernel variant, blocks per wave and grid from the autotuner, on this workload
    from paper_2604_07980_amd import autotune

    def run_batch():
        batch()
        return out_b
    table = autotune.tune(run_batch, p, reps=5, warmup=2)
    ms_batch = timed(batch)
    ocsr.reset_timing()
    ocsr.set_timing(True)
    for _ in range(steps):
        batch()
    torch.cuda.synchronize()
    ocsr.set_timing(False)
    kern = {}
    for name in ("census", "match", "match_far", "match_close", "aggregate"):
        cnt, tot = ocsr.kernel_time(name)
        if cnt:
            kern[name] = {"launches": cnt, "avg_us": round(1e3 * tot / cnt, 3)}
    # level pixels of the census tiles the call makes (those some box's search reads)
    census_px = sum(accounting.census_pixels(s.left.shape[1], s.left.shape[0],
                                             accounting.census_tiles(s.left.shape[1], s.left.shape[0],
                                                                     s.boxes, p), p)
                    for s in scenes)
    census_px_full = sum(2 * L.numel() + 2 * (L.shape[0] // p["close_scale"]) * (L.shape[1] // p["close_scale"])
                         for L, _ in imgs)
    costs_far = sum(w["costs_far"] for w in work)
    ops = {"census": census_px * 62, "match": costs * 4, "match_far": costs_far * 4,
           "match_close": (costs - costs_far) * 4}
    for k, v in ops.items():
        if k in kern:
            kern[k]["tops"] = round(v / (kern[k]["avg_us"] * 1e-6) / 1e12, 3)
            kern[k]["frac"] = round(kern[k]["tops"] / INT_PEAK_TOPS, 4)
    ms_frames = timed(per_frame)          # per-frame calls with the same tuned settings
    identical = bool(torch.equal(out_b, torch.cat(outs_f)))
    autotune.reset(p)
    return {"workload": "batch_16x1920x1200: 16 uint8 stereo pairs, min(128, Poisson(40)) boxes "
                        "per frame (log-uniform 12..512 px, overlaps occlude), params as the "
                        "realistic frame",
            "boxes": int(boxes.shape[0]), "blocks": sum(w["blocks"] for w in work),
            "census_level_px": census_px, "census_level_px_all_tiles": census_px_full,
            "costs_per_batch": costs, "steps": steps,
            "ms_per_batch": round(ms_batch, 4),
            "value": round(costs / (ms_batch * 1e-3) / 1e9, 3), "unit": "Gcost/s",
            "ms_per_batch_untuned": round(ms_default, 4),
            "autotune": {"variants": table.variants, "blocks_per_wave": table.blocks_per_wave,
                         "match_wgs_per_cu": table.match_wgs_per_cu},
            "kernels": kern,
            "ms_16_frame_calls": round(ms_frames, 4),
            "speedup_vs_16_calls": round(ms_frames / ms_batch, 3),
            "identical_to_16_calls": identical}


def dense_section(ocsr, L, R, steps, sparse_ms):
    """The dense counterpart on the same 1920x1080 pair: census of both views at full
    resolution, then every pixel over d = 0..191 with 5x5 summed Hamming costs, WTA in
    both views and the L/R check."""
    import torch
    W, H = L.shape[1], L.shape[0]
    ws = ocsr.Workspace()

    def run():
        CL, CR = ocsr.census_many([L, R], [1, 1])
        return ocsr.dense(CL, CR, 0, 191, 2, 1, workspace=ws)

    for _ in range(3):
        run()
    torch.cuda.synchronize()
    ocsr.reset_timing()
    ocsr.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        disp = run()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    ocsr.set_timing(False)
    kern = {}
    for name in ("census", "dense", "dense_check"):
        cnt, tot = ocsr.kernel_time(name)
        if cnt:
            kern[name] = {"launches": cnt, "avg_us": round(1e3 * tot / cnt, 3)}
    costs = W * H * 192
    if "dense" in kern:
        # 4 int32 ops per cost in each of the two views
        kern["dense"]["tops"] = round(2 * 4 * costs / (kern["dense"]["avg_us"] * 1e-6) / 1e12, 3)
    return {"workload": "dense_1080p: the realistic 1920x1080 pair, census 7x9 at s=1, "
                        "d = 0..191, 5x5 window, WTA left and right, L/R <= 1",
            "costs_per_frame": costs, "ms_per_frame": round(ms, 4),
            "value": round(costs / (ms * 1e-3) / 1e9, 3), "unit": "Gcost/s",
            "valid_fraction": round(float((disp >= 0).float().mean()), 4),
            "ms_sparse_frame": round(sparse_ms, 4),
            "dense_over_sparse_time": round(ms / sparse_ms, 2), "kernels": kern}


def rect_section(ocsr, synth, steps):
    """Auto-rectification offset search on the ground-like 1080p pair with its right view
    6 rows low: census of both views at s = 2, then the dense matcher (d 0..63, 5x5, L/R
    <= 1) on a 960 x 128 band of road rows for the 9 offsets -4..4, counts of d > 2, and
    the host filter. Kernel times from HIP events."""
    import torch
    dev = torch.device("cuda:0")
    left, right = synth.road_pair(drift=6)
    L = torch.from_numpy(left).to(dev)
    R = torch.from_numpy(right).to(dev)
    p = dict(roi_x0=0, roi_y0=300, roi_w=960, roi_h=128, delta_min=-4, delta_max=4, dmin=0,
             dmax=63, radius=2, lr_tol=1, d_min=2)
    ws = ocsr.Workspace()
    counts = torch.empty(9, dtype=torch.int32, device=dev)

    def run():
        CL, CR = ocsr.census_many([L, R], [2, 2])
        ocsr.rect_offset_counts(CL, CR, p, workspace=ws, counts=counts)

    for _ in range(3):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    ocsr.reset_timing()
    ocsr.set_timing(True)
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    ocsr.set_timing(False)
    kern = {}
    costs = 9 * p["roi_w"] * p["roi_h"] * (p["dmax"] - p["dmin"] + 1)
    for name in ("census", "rect_dense", "rect_count"):
        cnt, tot = ocsr.kernel_time(name)
        if cnt:
            kern[name] = {"avg_us": round(1e3 * tot / cnt, 3)}
    if "rect_dense" in kern:
        # 4 int32 ops per cost in each of the two views
        tops = 2 * MATCH_OPS_PER_COST * costs / (kern["rect_dense"]["avg_us"] * 1e-6) / 1e12
        kern["rect_dense"].update(tops=round(tops, 3), frac=round(tops / INT_PEAK_TOPS, 4))
    f = ocsr.RectFilter(5, 1)
    raw, filt = f.update(counts.cpu().numpy(), p["delta_min"])
    return {"workload": "road_1080p: ground-like 1920x1080 pair, right view 6 rows low; s=2, "
                        "ROI 960x128, offsets -4..4, dense d 0..63 5x5, count d > 2",
            "ms_per_frame": round(ms, 4), "costs_per_frame": costs,
            "gcost_per_s": round(costs / (ms * 1e-3) / 1e9, 3),
            "estimate_level_rows": raw, "first_filtered": filt, "kernels": kern}


def serving_section(ocsr, synth, n_requests, pool_size):
    """The serving workload: Poisson arrivals at 120/s mixing 1280x720, 1920x1080 and
    3840x2160 frames (0.3/0.5/0.2) from resident image pools, 1..200 boxes, close
    ranges 0..127/191/255; continuous batching under a 4 GiB budget. Also run with all
    requests arriving at once (throughput), and as plain per-frame calls one after
    another, whose outputs the served ones must equal."""
    import numpy as np
    import torch
    from paper_2604_07980_amd import serve
    dev = torch.device("cuda:0")
    pools = [[(torch.from_numpy(L).to(dev), torch.from_numpy(R).to(dev))
              for L, R in synth.serving_pool(res, pool_size, seed=5000 + k)]
             for k, res in enumerate(synth.SERVING_RESOLUTIONS)]
    spec = synth.serving_requests(n_requests, pool_sizes=(pool_size,) * 3)

    def requests(at_once):
        return [serve.Request(q["rid"], *pools[q["res"]][q["pool"]], q["boxes"], q["params"],
                              0.0 if at_once else q["arrival"]) for q in spec]

    def served(at_once):
        srv = serve.Server(serve.GpuExecutor(n_slots=3), mem_budget=4 << 30)
        t0 = time.perf_counter()
        res = srv.run(requests(at_once))
        wall = time.perf_counter() - t0
        return res, serve.summarize(res, wall)

    served(True)                                   # warm-up: kernels, pools, allocator
    res_rt, rt = served(False)
    res_sat, sat = served(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = []
    ws = ocsr.Workspace()
    for q in requests(True):
        out = ocsr.range_frame(q.left, q.right, torch.from_numpy(q.boxes).to(dev), q.params,
                               cap_blocks=1 << 18, workspace=ws)
        plain.append(ocsr.results_to_numpy(out))
    wall_plain = time.perf_counter() - t0
    identical = all((a.boxes.view(np.int32) == b.view(np.int32)).all() and
                    (c.boxes.view(np.int32) == b.view(np.int32)).all()
                    for a, c, b in zip(res_rt, res_sat, plain))
    r4 = lambda v: None if v is None else round(v, 4)
    return {"workload": f"serving mix: {n_requests} requests, Poisson 120/s, 1280x720 / 1920x1080 "
                        f"/ 3840x2160 (0.3/0.5/0.2), 1..200 boxes, close 0..127/191/255, "
                        f"{pool_size} resident pairs per resolution, 4 GiB budget, 3 streams",
            "realtime_120_per_s": {"frames_per_s": r4(rt["frames_per_s"]),
                                   "latency_ms": {k: r4(v) for k, v in rt["latency_ms"].items()},
                                   "mean_batch_frames": r4(rt["mean_batch_frames"])},
            "all_at_once": {"frames_per_s": r4(sat["frames_per_s"]),
                            "latency_ms": {k: r4(v) for k, v in sat["latency_ms"].items()},
                            "mean_batch_frames": r4(sat["mean_batch_frames"])},
            "plain_per_frame_calls": {"frames_per_s": r4(n_requests / wall_plain)},
            "identical_to_plain_calls": bool(identical)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path is per frame "
              "and shards by frames, see DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2604_07980_amd import accounting, ocsr, synth

    if args.copy_calibration > 0:
        # a buffer well beyond the 256 MB last-level cache, so the copy's reads come from
        # HBM; the source is filled first and not touched again before the copies
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.zeros_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 5}), flush=True)
        return

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sc = synth.scene_realistic()
    p = synth.params_for(2)
    H, W = sc.left.shape
    L = torch.from_numpy(sc.left).to(dev)
    R = torch.from_numpy(sc.right).to(dev)
    boxes = torch.from_numpy(sc.boxes).to(dev)
    n = boxes.shape[0]
    ocsr.set_fused(args.fused)
    ws = ocsr.Workspace()
    out = torch.empty((n, 8), dtype=torch.int32, device=dev)

    # work of one frame, from the library's own block records (outside the timed region)
    fw = frame_costs(ocsr, L, R, boxes, p)
    costs, costs_far, evals, nb = fw["costs"], fw["costs_far"], fw["evals"], fw["blocks"]
    census_px_full = 2 * (W * H) + 2 * (W // 2) * (H // 2)
    tiles = accounting.census_tiles(W, H, sc.boxes, p)
    tiles_all = accounting.census_tiles(W, H, sc.boxes, p, full=True)
    census_px = accounting.census_pixels(W, H, tiles, p)   # pixels of the tiles made
    census_bits = (2 * p["sx"] + 1) * (2 * p["sy"] + 1)

    def step():
        ocsr.range_frame(L, R, boxes, p, workspace=ws, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K back-to-back frames
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = 1e3 * (t1 - t0) / args.steps

    # the same K frames again with every kernel bracketed by HIP events on its stream
    ocsr.reset_timing()
    ocsr.set_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_per_step_events = 1e3 * (time.perf_counter() - t2) / args.steps
    ocsr.set_timing(False)
    kern = {}
    for name in ("census", "plan", "match", "match_far", "match_close", "aggregate", "reset",
                 "fused", "graph"):
        cnt, tot = ocsr.kernel_time(name)
        if cnt:
            kern[name] = {"launches": cnt, "avg_us": 1e3 * tot / cnt}

    # per-frame latency: enqueue to result on the host, one frame at a time
    lat = []
    for _ in range(args.latency_steps):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - a))
    lat = np.array(lat)

    # the same frame submitted as a replayed HIP graph (one submission per frame)
    ocsr.set_graph(True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_graph = 1e3 * (time.perf_counter() - t0) / args.steps
    glat = []
    for _ in range(args.latency_steps):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        glat.append(1e3 * (time.perf_counter() - a))
    ocsr.set_graph(False)
    glat = np.array(glat)

    # per-box 3D point and covariance from the frame's results (a step after the timed
    # path): kernel time from HIP events, outside the timed steps
    geom = synth.point_geometry(W, H, p)
    pts = ocsr.box_points(boxes, out, geom)
    ocsr.reset_timing()
    ocsr.set_timing(True)
    for _ in range(args.steps):
        ocsr.box_points(boxes, out, geom, out=pts)
    torch.cuda.synchronize()
    ocsr.set_timing(False)
    pcnt, ptot = ocsr.kernel_time("points")
    points = {"boxes": int(n), "valid": int(ocsr.points_to_numpy(pts)["valid"].sum()),
              "us_per_call": round(1e3 * ptot / max(pcnt, 1), 3)}

    # priority selection under a budget of 20 objects (a step before ranging): kernel time
    # on the frame's 64 boxes and on a 16-frame call of 1000 boxes each
    sel_out, sel_rank = ocsr.select_boxes([(W, H, n)], boxes, 20)
    rng = np.random.default_rng(77)
    bx0 = rng.integers(-80, W, 16000)
    by0 = rng.integers(-80, H, 16000)
    many = torch.from_numpy(np.stack([bx0, by0, bx0 + rng.integers(1, 400, 16000),
                                      by0 + rng.integers(1, 300, 16000), np.ones(16000, int)],
                                     1).astype(np.int32)).to(dev)
    many_out, many_rank = ocsr.select_boxes([(W, H, 1000)] * 16, many, 20)
    select = {"budget": 20}
    for key, frames_, bx, o, r in (("frame_64_boxes", [(W, H, n)], boxes, sel_out, sel_rank),
                                   ("16_frames_1000_boxes", [(W, H, 1000)] * 16, many, many_out,
                                    many_rank)):
        ocsr.reset_timing()
        ocsr.set_timing(True)
        for _ in range(args.steps):
            ocsr.select_boxes(frames_, bx, 20, out=o, rank=r)
        torch.cuda.synchronize()
        ocsr.set_timing(False)
        scnt, stot = ocsr.kernel_time("select")
        select[key] = {"us_per_call": round(1e3 * stot / max(scnt, 1), 3)}
    select["frame_64_boxes"]["kept"] = int(((sel_out[:, 4] & 1) == 1).sum().item())

    # algorithmic work per launch: census = informative comparisons (the centre term
    # is constant); match = 4 int32 ops per 64-bit Hamming cost
    census_ops = census_px * (census_bits - 1) * CENSUS_OPS_PER_CMP
    far_ops = costs_far * MATCH_OPS_PER_COST
    close_ops = (costs - costs_far) * MATCH_OPS_PER_COST
    work = {"census": census_ops, "match": far_ops + close_ops, "match_far": far_ops,
            "match_close": close_ops, "fused": census_ops + far_ops + close_ops}
    for k, ops in work.items():
        if k in kern:
            kern[k]["tops"] = ops / (kern[k]["avg_us"] * 1e-6) / 1e12
            kern[k]["frac"] = kern[k]["tops"] / INT_PEAK_TOPS
    dom = max((k for k in work if k in kern), key=lambda k: kern[k]["avg_us"])
    ach = kern[dom]["tops"]
    roofline = {"kernel": dom, "bound": "alu", "achieved": round(ach, 3), "peak": round(INT_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(ach / INT_PEAK_TOPS, 4),
                "traffic": measured_traffic(dom), "ops_per_launch": work[dom]}

    res = {
        "metric": METRIC,
        "value": round(costs / (ms_per_step * 1e-3) / 1e9, 3),
        "unit": "Gcost/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "realistic_1080p: one 1920x1080 uint8 stereo pair, 32 ranged boxes "
                               "(19 far 4x4 blocks d 0..31 at s=1, 13 close 8x8 blocks d 0..191 at "
                               "s=2) + 32 occluder boxes, census 7x9 on the tiles the searches read, "
                               "trimmed median",
                   "costs_per_frame": costs, "costs_far": costs_far,
                   "block_evals_per_frame": evals,
                   "blocks": int(nb), "census_level_px": census_px,
                   "census_tiles": len(tiles), "census_tiles_all": len(tiles_all),
                   "census_level_px_all_tiles": census_px_full},
        "block_evals_per_s": round(evals / (ms_per_step * 1e-3), 1),
        "ms_per_step_with_kernel_events": round(ms_per_step_events, 4),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "frames": int(len(lat))},
        "graph": {"ms_per_step": round(ms_graph, 4),
                  "latency_ms": {"p50": round(float(np.percentile(glat, 50)), 4),
                                 "p99": round(float(np.percentile(glat, 99)), 4)}},
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "roofline": roofline,
        "points": points,
        "select": select,
    }
    if args.vertical_steps > 0:
        res["vertical"] = vertical_section(ocsr, synth, args.vertical_steps, max(3, args.warmup // 10))
    if args.batch_steps > 0:
        res["batch"] = batch_section(ocsr, synth, args.batch_steps, max(3, args.warmup // 10))
    if args.rect_steps > 0:
        res["rect"] = rect_section(ocsr, synth, args.rect_steps)
    if args.dense_steps > 0:
        res["dense"] = dense_section(ocsr, L, R, args.dense_steps, ms_per_step)
    if args.serve_requests > 0:
        res["serving"] = serving_section(ocsr, synth, args.serve_requests, args.serve_pool)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(sc, p, costs, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
