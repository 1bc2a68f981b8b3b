"""The serving scheduler on a simulated executor and clock (no GPU): every request is
served once with its own results, batches never mix parameters or exceed 16 frames,
device memory in use never passes the budget, queued requests start as soon as a slot
and memory free up, and a request larger than the budget is refused alone."""
import numpy as np
import pytest

from paper_2604_07980_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def idle(self, ex):
        self.t = max(self.t, ex.next_done())


class FakeImage:
    def __init__(self, H, W):
        self.shape = (H, W)


class FakeExecutor:
    """Batch time = 1 ms + 0.5 ms per frame; memory = 1 MB per frame + 1 KB per box;
    a request's result is derived from its own boxes only."""

    def __init__(self, clock, n_slots=2):
        self.clock = clock
        self.n_slots = n_slots
        self.running = {}
        self.log = []              # (submit time, slot, [rids], bytes)

    def bytes_needed(self, reqs):
        return sum((1 << 20) + 1024 * len(r.boxes) for r in reqs)

    def submit(self, slot, reqs):
        assert slot not in self.running
        self.running[slot] = (self.clock.now() + 1e-3 + 0.5e-3 * len(reqs), reqs)
        self.log.append((self.clock.now(), slot, [r.rid for r in reqs], self.bytes_needed(reqs)))

    def poll(self, slot):
        return self.clock.now() >= self.running[slot][0]

    def collect(self, slot):
        _, reqs = self.running.pop(slot)
        return [r.boxes.sum(axis=1).astype(np.int64) for r in reqs]

    def next_done(self):
        return min(t for t, _ in self.running.values())


def _requests(n, seed=0, rate=2000.0, classes=2, max_boxes=20):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for rid in range(n):
        t += rng.exponential(1.0 / rate)
        nb = int(rng.integers(0, max_boxes + 1))
        boxes = rng.integers(0, 100, size=(nb, 5)).astype(np.int32)
        params = {"cls": int(rng.integers(0, classes))}
        out.append(serve.Request(rid, FakeImage(48, 64), FakeImage(48, 64), boxes, params, t))
    return out


def _run(reqs, budget=8 << 20, slots=2, max_frames=16):
    clock = FakeClock()
    ex = FakeExecutor(clock, slots)
    srv = serve.Server(ex, mem_budget=budget, max_frames=max_frames, clock=clock)
    return srv, ex, srv.run(reqs)


def test_every_request_served_once_with_its_own_result():
    reqs = _requests(300)
    srv, ex, res = _run(reqs)
    assert [r.rid for r in res] == list(range(300))
    for q, r in zip(reqs, res):
        assert r.error is None
        assert (r.boxes == q.boxes.sum(axis=1)).all()
        assert r.arrival <= r.start <= r.done
    assert sorted(rid for _, _, rids, _ in ex.log for rid in rids) == list(range(300))


def test_batches_are_homogeneous_and_bounded():
    reqs = _requests(400, rate=20000.0)
    srv, ex, res = _run(reqs, budget=64 << 20, max_frames=16)
    by_id = {q.rid: q for q in reqs}
    sizes = []
    for _, _, rids, _ in ex.log:
        assert len(rids) <= 16
        assert len({by_id[i].params["cls"] for i in rids}) == 1
        sizes.append(len(rids))
    assert max(sizes) > 1          # under load, queued requests do share batches


def test_memory_budget_never_exceeded():
    reqs = _requests(300, rate=50000.0, max_boxes=60)
    budget = 5 << 20
    srv, ex, res = _run(reqs, budget=budget, slots=4)
    # replay the submissions against completions to get the in-use profile
    assert srv.peak_in_use <= budget
    for _, _, _, nbytes in ex.log:
        assert nbytes <= budget
    assert srv.in_use == 0


def test_queued_requests_start_when_a_slot_frees():
    # two slots, everything arrives at once: the third batch starts exactly when the
    # first one completes
    reqs = [serve.Request(i, FakeImage(8, 8), FakeImage(8, 8), np.zeros((1, 5), np.int32),
                          {"cls": i % 3}, 0.0) for i in range(3)]
    srv, ex, res = _run(reqs, slots=2)
    starts = [t for t, _, _, _ in ex.log]
    assert starts[0] == starts[1] == 0.0
    assert starts[2] == pytest.approx(1.5e-3)


def test_oldest_request_always_in_the_next_batch():
    reqs = _requests(200, rate=30000.0)
    srv, ex, res = _run(reqs, slots=1)
    served = set()
    arrival = {q.rid: q.arrival for q in reqs}
    for t, _, rids, _ in ex.log:
        waiting = [q.rid for q in reqs if q.rid not in served and arrival[q.rid] <= t]
        assert min(waiting) in rids
        served.update(rids)


def test_request_over_budget_is_refused_alone():
    reqs = _requests(20)
    big = serve.Request(99, FakeImage(8, 8), FakeImage(8, 8), np.zeros((5000, 5), np.int32),
                        {"cls": 0}, 0.001)
    srv, ex, res = _run(reqs + [big], budget=2 << 20)
    by = {r.rid: r for r in res}
    assert by[99].error is not None and by[99].boxes is None
    assert all(by[q.rid].error is None for q in reqs)


def test_summary():
    reqs = _requests(50)
    srv, ex, res = _run(reqs)
    s = serve.summarize(res, wall=res[-1].done)
    assert s["served"] == 50 and s["rejected"] == 0
    assert s["latency_ms"]["p50"] <= s["latency_ms"]["p99"]


def test_cancelled_while_queued_is_never_submitted():
    # one slot, three requests at t = 0: the second is cancelled at 0.2 ms, while the
    # first runs (1.5 ms), so it leaves the queue and the third runs next
    reqs = [serve.Request(i, FakeImage(8, 8), FakeImage(8, 8), np.zeros((1, 5), np.int32),
                          {"cls": i}, 0.0) for i in range(3)]
    reqs[1].cancel_at = 0.2e-3
    srv, ex, res = _run(reqs, slots=1)
    assert res[1].error == serve.ERR_CANCELLED and res[1].boxes is None
    submitted = [rid for _, _, rids, _ in ex.log for rid in rids]
    assert submitted == [0, 2]
    assert ex.log[1][0] == pytest.approx(1.5e-3)      # the third starts when the slot frees


def test_cancelled_while_running_discards_its_result():
    reqs = [serve.Request(0, FakeImage(8, 8), FakeImage(8, 8), np.zeros((1, 5), np.int32),
                        {"cls": 0}, 0.0, cancel_at=1e-3)]
    srv, ex, res = _run(reqs, slots=1)
    assert [rid for _, _, rids, _ in ex.log for rid in rids] == [0]
    assert res[0].error == serve.ERR_CANCELLED and res[0].boxes is None
    assert srv.in_use == 0


def test_deadline_times_out_queued_requests_only():
    # one slot, batches of one frame: request 0 runs 0..1.5 ms; request 1 (deadline 1 ms)
    # is still queued then and times out; request 2 (deadline 2 ms) starts at 1.5 ms and
    # is served even though it completes after its deadline
    reqs = [serve.Request(i, FakeImage(8, 8), FakeImage(8, 8), np.zeros((1, 5), np.int32),
                          {"cls": 0}, 0.0) for i in range(3)]
    reqs[1].deadline = 1e-3
    reqs[2].deadline = 2e-3
    srv, ex, res = _run(reqs, slots=1, max_frames=1)
    assert res[1].error == serve.ERR_DEADLINE
    assert res[0].error is None and res[2].error is None
    assert res[2].done > 2e-3
    assert [rid for _, _, rids, _ in ex.log for rid in rids] == [0, 2]


def test_waiting_request_times_out_without_other_events():
    # the only queued request cannot fit while a larger one runs; its deadline passes
    # while the clock idles on the running batch
    reqs = [serve.Request(0, FakeImage(8, 8), FakeImage(8, 8), np.zeros((1000, 5), np.int32),
                          {"cls": 0}, 0.0),
            serve.Request(1, FakeImage(8, 8), FakeImage(8, 8), np.zeros((1000, 5), np.int32),
                          {"cls": 1}, 0.0, deadline=0.5e-3)]
    srv, ex, res = _run(reqs, budget=3 << 20, slots=2)
    assert res[1].error == serve.ERR_DEADLINE
    assert res[0].error is None
