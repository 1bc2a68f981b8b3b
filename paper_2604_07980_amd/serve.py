"""Serving loop for ranging requests on one GPU: continuous batching under a device-memory
budget.

A request is one stereo frame (left/right uint8 images already in device memory) with
its detection boxes (host int32 [n, 5]) and matching parameters. Requests enter a queue
at their arrival time. Whenever an execution slot (a stream with its own resident
memory) is free, the server forms a batch from the queue -- the oldest request, then
later queued requests with the same parameters, up to 16 frames -- provided its device
memory (workspace with the descriptor images, boxes, results) fits the slot and what the
budget has left, and submits it on the slot's stream. Batches on different slots overlap
on the device; a slot is reaped as soon as its batch completes, its memory returns to
the budget, and queued requests are admitted into the next batch without waiting for
the others. Each request's results do not depend on which batch it ran in: frames of a
batch share no state.

A request may carry a deadline (it times out if it is still queued then) and a
cancellation time (it leaves the queue then, or, already submitted, its results are
discarded when its batch completes).

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
BOX_BUCKETS = (16, 64, 256, 1024)     # box capacities of the per-frame graphs

ERR_BUDGET = "request exceeds the device-memory budget"
ERR_DEADLINE = "deadline passed before the request was admitted"
ERR_CANCELLED = "cancelled"


@dataclass
class Request:
    rid: int
    left: object            # uint8 [H, W] device tensor (or any image handle the executor takes)
    right: object
    boxes: np.ndarray       # int32 [n, 5], host
    params: dict
    arrival: float = 0.0    # seconds from the start of the stream
    deadline: float | None = None    # still queued at this time: times out
    cancel_at: float | None = None   # the client cancels at this time

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
        # the most one slot can hold (executors with fixed per-slot memory)
        cap = getattr(executor, "slot_capacity", None)
        self.slot_cap = min(self.budget, int(cap())) if cap is not None else self.budget

    def _fits(self, need: int) -> bool:
        return need <= self.slot_cap and self.in_use + need <= self.budget

    def _form_batch(self, queue: collections.deque):
        """The oldest queued request and later ones with its parameters, while the
        batch's memory fits the slot and the budget left. Returns (requests, bytes) or
        None."""
        head = queue[0]
        key = params_key(head.params)
        batch = [head]
        need = self.ex.bytes_needed(batch)
        if not self._fits(need):
            return None
        for r in list(queue)[1:]:
            if len(batch) == self.max_frames:
                break
            if params_key(r.params) != key:
                continue
            trial = self.ex.bytes_needed(batch + [r])
            if not self._fits(trial):
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
                if self.ex.bytes_needed([r]) > self.slot_cap:
                    results.append(Result(r.rid, None, r.arrival, now, now, 0, error=ERR_BUDGET))
                else:
                    queue.append(r)
                progressed = True
            # queued requests cancelled or past their deadline leave the queue
            if queue and any(r.cancel_at is not None or r.deadline is not None for r in queue):
                keep = collections.deque()
                for r in queue:
                    if r.cancel_at is not None and r.cancel_at <= now:
                        results.append(Result(r.rid, None, r.arrival, now, now, 0, error=ERR_CANCELLED))
                    elif r.deadline is not None and r.deadline < now:
                        results.append(Result(r.rid, None, r.arrival, now, now, 0, error=ERR_DEADLINE))
                    else:
                        keep.append(r)
                if len(keep) != len(queue):
                    progressed = True
                queue = keep
            for s in list(busy):
                if self.ex.poll(s):
                    sl = busy.pop(s)
                    done = self.clock.now()
                    for r, out in zip(sl.reqs, self.ex.collect(s)):
                        if r.cancel_at is not None and r.cancel_at <= done:
                            # cancelled while on the device: its results are discarded
                            results.append(Result(r.rid, None, r.arrival, sl.start, done,
                                                  len(sl.reqs), error=ERR_CANCELLED))
                        else:
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
                t = pending[0].arrival
                for r in queue:   # a queued request that can only wait may still time out
                    for ev in (r.cancel_at, r.deadline):
                        if ev is not None:
                            t = min(t, ev)
                self.clock.wait_until(t)
            elif queue:
                # nothing runs and the head does not fit: only a deadline or cancellation
                # can change that (requests larger than a slot are refused on arrival)
                evs = [ev for r in queue for ev in (r.cancel_at, r.deadline) if ev is not None]
                if not evs:
                    raise RuntimeError("queued requests can never be admitted")
                self.clock.wait_until(min(evs) + 1e-9)
        results.sort(key=lambda r: r.rid)
        return results


def _align(v: int, a: int = 256) -> int:
    return (v + a - 1) // a * a


def _bucket(n: int) -> int | None:
    for b in BOX_BUCKETS:
        if n <= b:
            return b
    return None


class GpuExecutor:
    """Runs batches on one stream per slot (default stream priority), each slot with a
    resident arena of `slot_bytes` of device memory allocated once, at construction:
    the workspace (descriptor images and matching state), boxes and results of a batch
    are carved from it, so serving allocates no device memory. Box lists are staged
    through per-slot pinned host memory.

    A batch of several frames runs as one ocsr_range_batch call. A batch of one frame,
    with `graphs` on, runs as the replay of a HIP graph captured per slot and per
    (resolution, box capacity, parameters) bucket: the frame's images are copied into the
    slot's staging images and its boxes padded to the bucket's capacity with empty boxes
    that are not ranged (they occlude nothing), so every replay finds its inputs at the
    captured addresses. With max_objects set, each frame's boxes first go through the
    priority selection (ocsr_select_boxes): candidates past the budget keep occluding
    but are not ranged (reason NOT_RANGED)."""

    def __init__(self, n_slots: int = 3, device: str = "cuda:0", cap_blocks: int = 1 << 18,
                 slot_bytes: int = 1280 << 20, graphs: bool = False,
                 max_objects: int | None = None, crop_permille=None):
        import torch
        from . import ocsr
        self.torch, self.ocsr = torch, ocsr
        self.dev = torch.device(device)
        self.n_slots = n_slots
        self.cap_blocks = cap_blocks
        self.slot_bytes = int(slot_bytes)
        self.graphs = graphs
        self.max_objects = max_objects
        self.crop = tuple(crop_permille) if crop_permille is not None else ocsr.DEFAULT_CROP_PERMILLE
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(n_slots)]
        self.arenas = [torch.empty(self.slot_bytes + 256, dtype=torch.uint8, device=self.dev)
                       for _ in range(n_slots)]
        self.base = [(-a.data_ptr()) % 256 for a in self.arenas]
        self.pinned = [None] * n_slots
        self.events = [None] * n_slots
        self.outs = [None] * n_slots
        self.reqs = [None] * n_slots
        self.graph_frames = 0

    def slot_capacity(self) -> int:
        return self.slot_bytes

    # -- memory layout of a batch in a slot's arena --------------------------------
    def _single_graph(self, reqs) -> bool:
        return self.graphs and len(reqs) == 1 and _bucket(len(reqs[0].boxes)) is not None

    def _layout(self, reqs):
        """Byte offsets and sizes of (workspace, boxes, results, selected boxes, ranks,
        staging images) for a batch, and the total."""
        if self._single_graph(reqs):
            H, W = reqs[0].shape
            nb = _bucket(len(reqs[0].boxes))
            ws = self.ocsr.frame_workspace_bytes(W, H, reqs[0].params, nb, self.cap_blocks)
            stage = 2 * _align(H * W)
        else:
            shapes = [(r.shape[0], r.shape[1], len(r.boxes)) for r in reqs]
            nb = sum(len(r.boxes) for r in reqs)
            ws = self.ocsr.batch_workspace_bytes(shapes, reqs[0].params, self.cap_blocks)
            stage = 0
        sel = self.max_objects is not None
        sizes = [_align(ws), _align(nb * 20), _align(nb * 32), _align(nb * 20) if sel else 0,
                 _align(nb * 4) if sel else 0, stage]
        offs, at = [], 0
        for sz in sizes:
            offs.append(at)
            at += sz
        return offs, sizes, at, nb

    def bytes_needed(self, reqs) -> int:
        return self._layout(reqs)[2]

    def _region(self, slot, off, nbytes):
        b = self.base[slot] + off
        return self.arenas[slot][b:b + nbytes]

    def submit(self, slot: int, reqs) -> None:
        torch, ocsr = self.torch, self.ocsr
        offs, sizes, total, nb = self._layout(reqs)
        if total > self.slot_bytes:
            raise ValueError(f"batch needs {total} bytes > the slot's {self.slot_bytes}")
        s = self.streams[slot]
        single = self._single_graph(reqs)
        host = np.zeros((nb, 5), np.int32)
        at = 0
        for r in reqs:
            host[at:at + len(r.boxes)] = r.boxes.reshape(-1, 5)
            at += len(r.boxes)
        # per-slot pinned staging of the box list (grown when a larger list comes; the
        # slot's previous batch was collected, so its copy is done)
        if self.pinned[slot] is None or self.pinned[slot].shape[0] < nb:
            self.pinned[slot] = torch.empty((max(nb, 256), 5), dtype=torch.int32).pin_memory()
        pin = self.pinned[slot][:nb]
        pin.copy_(torch.from_numpy(host))
        boxes = self._region(slot, offs[1], nb * 20).view(torch.int32).view(nb, 5)
        out = self._region(slot, offs[2], nb * 32).view(torch.int32).view(nb, 8)
        ws = ocsr.Workspace(self._region(slot, offs[0], sizes[0]))
        with torch.cuda.stream(s):
            boxes.copy_(pin, non_blocking=True)
            ranged = boxes
            if nb > 0 and self.max_objects is not None:
                sel = self._region(slot, offs[3], nb * 20).view(torch.int32).view(nb, 5)
                rank = self._region(slot, offs[4], nb * 4).view(torch.int32)
                counts = [nb] if single else [len(r.boxes) for r in reqs]   # padding included
                ranged, _ = ocsr.select_boxes([(r.shape[1], r.shape[0], c) for r, c in zip(reqs, counts)],
                                              boxes, self.max_objects, self.crop, out=sel, rank=rank)
            if single:
                H, W = reqs[0].shape
                Ls = self._region(slot, offs[5], H * W).view(H, W)
                Rs = self._region(slot, offs[5] + _align(H * W), H * W).view(H, W)
                Ls.copy_(reqs[0].left, non_blocking=True)
                Rs.copy_(reqs[0].right, non_blocking=True)
                ocsr.set_graph(True, self.dev.index)
                try:
                    ocsr.range_frame(Ls, Rs, ranged, reqs[0].params, cap_blocks=self.cap_blocks,
                                     workspace=ws, out=out)
                finally:
                    ocsr.set_graph(False, self.dev.index)
                self.graph_frames += 1
            elif nb > 0:
                frames = [(r.left, r.right, len(r.boxes)) for r in reqs]
                ocsr.range_batch(frames, ranged, reqs[0].params, cap_blocks=self.cap_blocks,
                                 workspace=ws, out=out)
            ev = torch.cuda.Event()
            ev.record(s)
        self.events[slot], self.outs[slot], self.reqs[slot] = ev, out, reqs

    def poll(self, slot: int) -> bool:
        return self.events[slot].query()

    def collect(self, slot: int) -> list[np.ndarray]:
        self.events[slot].synchronize()
        res = self.outs[slot].cpu().numpy().view(self.ocsr.BOX_RESULT_DTYPE).reshape(-1)
        out, off = [], 0
        for r in self.reqs[slot]:
            out.append(res[off:off + len(r.boxes)].copy())
            off += len(r.boxes)
        self.events[slot] = self.outs[slot] = self.reqs[slot] = None
        return out

    def graph_stats(self) -> dict:
        hits, builds = self.ocsr.graph_stats(self.dev.index)
        return {"graph_frames": self.graph_frames, "replays": hits, "captures": builds}


def summarize(results: list[Result], wall: float) -> dict:
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    return {"requests": len(results), "served": len(ok), "rejected": len(results) - len(ok),
            "frames_per_s": len(ok) / wall if wall > 0 else 0.0,
            "latency_ms": {"p50": float(np.percentile(lat, 50)) if len(lat) else None,
                           "p99": float(np.percentile(lat, 99)) if len(lat) else None},
            "mean_batch_frames": float(np.mean([r.batch_frames for r in ok])) if ok else 0.0}
