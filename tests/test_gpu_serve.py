"""Served requests (continuous batching over several streams, memory budget) give, bit
for bit, the results each request gets alone, and the oracle's."""
import numpy as np
import pytest
import torch

from paper_2604_07980_amd import serve, synth
from test_gpu_parity import assert_results_match, _cuda

pytestmark = pytest.mark.gpu

RES = ((96, 128), (120, 200), (160, 256))


def _stream(n, seed=77, rate=4000.0):
    pools = [[(_cuda(L), _cuda(R), L, R) for L, R in synth.serving_pool(res, 2, seed=seed + k)]
             for k, res in enumerate(RES)]
    rng = np.random.default_rng(seed)
    t, reqs, host = 0.0, [], {}
    for rid in range(n):
        t += float(rng.exponential(1.0 / rate))
        ri = int(rng.integers(0, len(RES)))
        H, W = RES[ri]
        nb = int(rng.integers(1, 26))
        planes = synth.random_boxes(rng, H, W, nb, scale=W / 1920, tau_s=64 * W / 1920)
        boxes = np.array([[p[0], p[1], p[2], p[3], synth.BOX_RANGE] for p in planes], np.int32)
        p = synth.params_for(5, width=W)
        p["close"] = dict(p["close"], dmax=int(rng.choice([63, 95, 127])))
        L, R, Lh, Rh = pools[ri][int(rng.integers(0, 2))]
        reqs.append(serve.Request(rid, L, R, boxes, p, t))
        host[rid] = (Lh, Rh)
    return reqs, host


def test_served_equals_alone_and_oracle(lib, orc):
    # arrivals 1 us apart: requests queue behind the first batches whatever the GPU's
    # speed, so batches of several frames must form
    reqs, host = _stream(60, rate=1e6)
    ex = serve.GpuExecutor(n_slots=3)
    budget = 3 * ex.bytes_needed(reqs[:8])
    srv = serve.Server(ex, mem_budget=budget)
    res = srv.run(reqs)
    assert [r.rid for r in res] == [q.rid for q in reqs]
    assert srv.peak_in_use <= budget and srv.in_use == 0
    assert max(r.batch_frames for r in res) > 1          # requests did share batches
    for q, r in zip(reqs, res):
        assert r.error is None
        alone = lib.results_to_numpy(lib.range_frame(q.left, q.right, _cuda(q.boxes), q.params))
        assert (alone.view(np.int32) == r.boxes.view(np.int32)).all(), q.rid
    for q in reqs[::7]:
        Lh, Rh = host[q.rid]
        want = orc.run_scene(Lh, Rh, q.params, q.boxes)[1][0]
        assert_results_match(res[q.rid].boxes, want)


def test_budget_refuses_oversized_request(lib):
    reqs, _ = _stream(6)
    ex = serve.GpuExecutor(n_slots=2)
    budget = max(ex.bytes_needed([q]) for q in reqs[1:])
    big = reqs[0]
    big.boxes = np.concatenate([big.boxes] * 2000)
    srv = serve.Server(ex, mem_budget=budget)
    res = srv.run(reqs)
    assert res[0].error is not None
    assert all(r.error is None for r in res[1:])


def test_served_with_object_budget(lib, orc):
    """With a per-frame budget the executor selects before ranging: every served result
    equals the oracle's on the oracle's own selection of that request's boxes."""
    reqs, host = _stream(30, seed=91)
    ex = serve.GpuExecutor(n_slots=2, max_objects=6)
    srv = serve.Server(ex, mem_budget=4 << 30)
    res = srv.run(reqs)
    n_dropped = 0
    for q in reqs[::3]:
        Lh, Rh = host[q.rid]
        H, W = Lh.shape
        sel, rank = orc.select_boxes(q.boxes, W, H, 6, lib.DEFAULT_CROP_PERMILLE)
        want = orc.run_scene(Lh, Rh, q.params, sel)[1][0]
        assert_results_match(res[q.rid].boxes, want)
        n_dropped += int((rank >= 6).sum())
    assert n_dropped > 0                                   # the budget did bind


def test_served_with_per_frame_graphs(lib, orc):
    """Single-frame batches replay a graph captured per slot and per (resolution, box
    capacity, parameters) bucket, with the frame's images copied into the slot's staging
    images and its boxes padded with empty, not-ranged boxes: every result equals the
    request run alone, and later frames of a bucket replay instead of capturing."""
    reqs, host = _stream(40, seed=123, rate=300.0)
    ex = serve.GpuExecutor(n_slots=2, graphs=True, slot_bytes=256 << 20)
    srv = serve.Server(ex, mem_budget=512 << 20)
    res = srv.run(reqs)
    st = ex.graph_stats()
    assert st["graph_frames"] > 0 and st["replays"] > 0
    for q, r in zip(reqs, res):
        assert r.error is None
        alone = lib.results_to_numpy(lib.range_frame(q.left, q.right, _cuda(q.boxes), q.params))
        assert (alone.view(np.int32) == r.boxes.view(np.int32)).all(), q.rid
    for q in reqs[::9]:
        Lh, Rh = host[q.rid]
        assert_results_match(res[q.rid].boxes, orc.run_scene(Lh, Rh, q.params, q.boxes)[1][0])


def test_deadline_and_cancellation_on_the_device(lib):
    """A request cancelled while its batch runs comes back as cancelled; one whose
    deadline passes while it waits for a slot times out; the rest are served."""
    reqs, _ = _stream(12, seed=5, rate=1e6)
    reqs[3].cancel_at = 0.0          # cancelled from the start: never submitted
    for q in reqs[6:]:
        q.deadline = 0.0             # all arrive at once behind one slot: most time out
    ex = serve.GpuExecutor(n_slots=1, slot_bytes=256 << 20)
    srv = serve.Server(ex, mem_budget=512 << 20, max_frames=1)
    res = srv.run(reqs)
    assert res[3].error == serve.ERR_CANCELLED and res[3].boxes is None
    assert any(r.error == serve.ERR_DEADLINE for r in res[6:])
    assert all(r.error is None for i, r in enumerate(res[:6]) if i != 3)
