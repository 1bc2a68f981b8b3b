"""Serving loop for ranging requests on one GPU: continuous batching under a device-memory
budget.

A request is one stereo frame (left/right uint8 images already in device memory) with
its detection boxes (host int32 [n, 5]) and matching parameters. Requests enter a queue
at their arrival time. Whenever an execution slot (a stream with its own workspace) is
free, the server forms a batch from the queue -- the oldest request, then later queued
requests with the same parameters, up to 16 frames -- provided its device memory
(workspace with the descriptor images, boxes, results) fits in what the budget has
left, and submits it as one ocsr_range_batch call on the slot's stream. Batches on
different slots overlap on the device; a slot is reaped as soon as its batch completes,
its memory returns to the budget, and queued requests are admitted into the next batch
without waiting for the others. Each request's results do not depend on which batch it
ran in: frames of a batch share no state.

The scheduler talks to an executor (GpuExecutor here; tests use a simulated one) and a
clock, so its policy can be checked without a device.
"""
from __future__ import annotations

import collections
import json
import time
from dataclasses import dataclass, field

import numpy as np

MAX_BATCH_FRAMES = 16


@dataclass
class Request:
    rid: int
    left: object            # uint8 [H, W] device tensor (or any image handle the executor takes)
    right: object
    boxes: np.ndarray       # int32 [n, 5], host
    params: dict
    arrival: float = 0.0    # seconds from the start of the stream

    @property
    def shape(self):
        return tuple(self.left.shape)


@dataclass
class Result:
    rid: int
    boxes: np.ndarray | None     # structured per-box results (None on error)
    arrival: float
    start: float
    done: float
    batch_frames: int
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def params_key(p: dict) -> str:
    return json.dumps(p, sort_keys=True)


class RealClock:
    """Wall clock; idle() yields the host thread while the device works (a timed sleep
    would oversleep by tens of microseconds and add that to every result's latency)."""

    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float) -> None:
        # sleep most of the way, then yield until the time is reached
        dt = t - self.now()
        if dt > 5e-4:
            time.sleep(dt - 3e-4)
        while self.now() < t:
            time.sleep(0)

    def idle(self, executor) -> None:
        time.sleep(0)


@dataclass
class _Slot:
    reqs: list = field(default_factory=list)
    nbytes: int = 0
    start: float = 0.0


class Server:
    """Continuous-batching scheduler over an executor's slots."""

    def __init__(self, executor, mem_budget: int = 4 << 30, max_frames: int = MAX_BATCH_FRAMES,
                 clock=None):
        if not 1 <= max_frames <= MAX_BATCH_FRAMES:
            raise ValueError(f"max_frames outside 1..{MAX_BATCH_FRAMES}")
        self.ex = executor
        self.budget = int(mem_budget)
        self.max_frames = max_frames
        self.clock = clock or RealClock()
        self.in_use = 0
        self.peak_in_use = 0
        self.batches = 0

    def _form_batch(self, queue: collections.deque):
        """The oldest queued request and later ones with its parameters, while the
        batch's memory fits the budget left. Returns (requests, bytes) or None."""
        head = queue[0]
        key = params_key(head.params)
        batch = [head]
        need = self.ex.bytes_needed(batch)
        if self.in_use + need > self.budget:
            return None
        for r in list(queue)[1:]:
            if len(batch) == self.max_frames:
                break
            if params_key(r.params) != key:
                continue
            trial = self.ex.bytes_needed(batch + [r])
            if self.in_use + trial > self.budget:
                break
            batch.append(r)
            need = trial
        return batch, need

    def run(self, requests) -> list[Result]:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: collections.deque = collections.deque()
        free = list(range(self.ex.n_slots))
        busy: dict[int, _Slot] = {}
        results: list[Result] = []
        while pending or queue or busy:
            progressed = False
            now = self.clock.now()
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                if self.ex.bytes_needed([r]) > self.budget:
                    results.append(Result(r.rid, None, r.arrival, now, now, 0,
                                          error="request exceeds the device-memory budget"))
                else:
                    queue.append(r)
                progressed = True
            for s in list(busy):
                if self.ex.poll(s):
                    sl = busy.pop(s)
                    done = self.clock.now()
                    for r, out in zip(sl.reqs, self.ex.collect(s)):
                        results.append(Result(r.rid, out, r.arrival, sl.start, done, len(sl.reqs)))
                    self.in_use -= sl.nbytes
                    free.append(s)
                    progressed = True
            while free and queue:
                fb = self._form_batch(queue)
                if fb is None:
                    break            # wait for memory to come back
                batch, nbytes = fb
                ids = {id(r) for r in batch}
                queue = collections.deque(r for r in queue if id(r) not in ids)
                s = free.pop(0)
                start = self.clock.now()
                self.ex.submit(s, batch)
                busy[s] = _Slot(batch, nbytes, start)
                self.in_use += nbytes
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                self.batches += 1
                progressed = True
            if progressed:
                continue
            if busy:
                self.clock.idle(self.ex)
            elif pending:
                self.clock.wait_until(pending[0].arrival)
        results.sort(key=lambda r: r.rid)
        return results


class GpuExecutor:
    """Runs batches with ocsr_range_batch, one stream per slot (default stream priority).
    A batch's workspace, boxes and results are allocated when it is submitted and
    released when it is collected, so the memory the server accounts for is what the
    batches in flight hold (allocations come from the framework's caching allocator).
    Box lists are staged through pinned host memory. With max_objects set, each frame's
    boxes first go through the priority selection (ocsr_select_boxes): candidates past
    the budget keep occluding but are not ranged (reason NOT_RANGED)."""

    def __init__(self, n_slots: int = 3, device: str = "cuda:0", cap_blocks: int = 1 << 18,
                 max_objects: int | None = None, crop_permille=None):
        import torch
        from . import ocsr
        self.torch, self.ocsr = torch, ocsr
        self.dev = torch.device(device)
        self.n_slots = n_slots
        self.cap_blocks = cap_blocks
        self.max_objects = max_objects
        self.crop = tuple(crop_permille) if crop_permille is not None else ocsr.DEFAULT_CROP_PERMILLE
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(n_slots)]
        self.events = [None] * n_slots
        self.outs = [None] * n_slots
        self.reqs = [None] * n_slots
        self.keep = [None] * n_slots

    def bytes_needed(self, reqs) -> int:
        shapes = [(r.shape[0], r.shape[1], len(r.boxes)) for r in reqs]
        nb = sum(len(r.boxes) for r in reqs)
        sel = nb * (5 * 4 + 4) if self.max_objects is not None else 0   # selected boxes, ranks
        return (self.ocsr.batch_workspace_bytes(shapes, reqs[0].params, self.cap_blocks)
                + nb * (5 * 4 + 8 * 4) + sel)

    def submit(self, slot: int, reqs) -> None:
        torch, ocsr = self.torch, self.ocsr
        s = self.streams[slot]
        boxes_h = torch.from_numpy(np.ascontiguousarray(
            np.concatenate([r.boxes.reshape(-1, 5) for r in reqs]).astype(np.int32))).pin_memory()
        with torch.cuda.stream(s):
            boxes = boxes_h.to(self.dev, non_blocking=True)
            out = torch.empty((boxes.shape[0], 8), dtype=torch.int32, device=self.dev)
            frames = [(r.left, r.right, len(r.boxes)) for r in reqs]
            ws = ocsr.Workspace()
            boxes_in = boxes
            if boxes.shape[0] > 0 and self.max_objects is not None:
                boxes, _ = ocsr.select_boxes([(r.shape[1], r.shape[0], len(r.boxes)) for r in reqs],
                                             boxes_in, self.max_objects, self.crop)
            if boxes.shape[0] > 0:
                ocsr.range_batch(frames, boxes, reqs[0].params, cap_blocks=self.cap_blocks,
                                 workspace=ws, out=out)
            ev = torch.cuda.Event()
            ev.record(s)
        self.events[slot], self.outs[slot], self.reqs[slot] = ev, out, reqs
        self.keep[slot] = (boxes_h, boxes_in, boxes, ws)   # held until the batch is collected

    def poll(self, slot: int) -> bool:
        return self.events[slot].query()

    def collect(self, slot: int) -> list[np.ndarray]:
        self.events[slot].synchronize()
        res = self.outs[slot].cpu().numpy().view(self.ocsr.BOX_RESULT_DTYPE).reshape(-1)
        out, off = [], 0
        for r in self.reqs[slot]:
            out.append(res[off:off + len(r.boxes)].copy())
            off += len(r.boxes)
        self.events[slot] = self.outs[slot] = self.reqs[slot] = self.keep[slot] = None
        return out


def summarize(results: list[Result], wall: float) -> dict:
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    return {"requests": len(results), "served": len(ok), "rejected": len(results) - len(ok),
            "frames_per_s": len(ok) / wall if wall > 0 else 0.0,
            "latency_ms": {"p50": float(np.percentile(lat, 50)) if len(lat) else None,
                           "p99": float(np.percentile(lat, 99)) if len(lat) else None},
            "mean_batch_frames": float(np.mean([r.batch_frames for r in ok])) if ok else 0.0}
