"""Continuous-batching request loop for the P2S simulator.

Requests (an image, D/r0 and a seed each) arrive over time.  The engine keeps
the basis and network resident, carves every batch's workspace (fields,
weights, blurred image, plan) out of one pre-allocated device arena, and
admits queued requests first come, first served whenever

  * one of `n_slots` batch slots is free (each slot is a HIP stream, so up to
    n_slots batches run on the device at once and new work overlaps work
    already in flight), and
  * the arena can hold the batch's workspace and the HBM budget (arena bytes
    in use plus the outputs of requests not yet finished) stays within
    `budget_bytes`.

It never waits to fill a batch: whatever is queued and fits goes out as soon as
a slot frees up.  A request whose frame alone cannot fit the budget is
rejected.  A batch whose launch fails (for example an allocation or launch
error from the library) fails only its own requests: their arena block is
returned and the loop keeps serving the others.

Images and outputs are the caller's device buffers, as in the C ABI; the
budget bounds what the engine itself holds on the device (the arena with the
plans and intermediates of the batches in flight) plus any output bytes an
executor reports for outputs it allocates itself.

Latency is finish time minus arrival time, both on the engine's host clock:
a batch counts as finished at the first poll that sees its completion event.

The engine talks to an executor (launch a batch on a slot, ask whether it has
finished, release it), so that the host logic runs unchanged against a fake
executor on the CPU and against the GPU executor, which drives the batched
C-ABI (p2s_batch_*).
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

ALIGN = 256


def _align(n: int) -> int:
    return (n + ALIGN - 1) // ALIGN * ALIGN


class Arena:
    """First-fit allocator of [0, capacity) in 256-byte units; adjacent free
    blocks are merged on release."""

    def __init__(self, capacity: int):
        self.capacity = capacity - capacity % ALIGN
        self.free_blocks: List[Tuple[int, int]] = [(0, self.capacity)] if self.capacity > 0 else []
        self.used: Dict[int, int] = {}

    @property
    def bytes_in_use(self) -> int:
        return sum(self.used.values())

    def alloc(self, n: int) -> Optional[int]:
        n = _align(max(n, 1))
        for i, (off, size) in enumerate(self.free_blocks):
            if size >= n:
                if size == n:
                    self.free_blocks.pop(i)
                else:
                    self.free_blocks[i] = (off + n, size - n)
                self.used[off] = n
                return off
        return None

    def release(self, off: int) -> None:
        n = self.used.pop(off)
        blocks = self.free_blocks
        blocks.append((off, n))
        blocks.sort()
        merged: List[Tuple[int, int]] = []
        for o, s in blocks:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free_blocks = merged


@dataclass
class Request:
    rid: int
    image: object                 # device tensor [C][H][W] (GPU executor) or a shape tuple (fake)
    d_over_r0: float
    seed: int
    arrival: float                # seconds on the engine clock
    shape: Tuple[int, int, int] = (0, 0, 0)
    out: object = None
    admitted: Optional[float] = None
    finished: Optional[float] = None
    batch_id: Optional[int] = None
    rejected: bool = False
    failed: bool = False
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


@dataclass
class _InFlight:
    batch_id: int
    slot: int
    requests: List[Request]
    handle: object
    arena_off: int
    arena_bytes: int
    out_bytes: int


class Engine:
    def __init__(self, executor, budget_bytes: int, n_slots: int = 2, max_batch_frames: int = 32,
                 clock: Optional[Callable[[], float]] = None):
        if n_slots < 1 or max_batch_frames < 1:
            raise ValueError("n_slots and max_batch_frames must be >= 1")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.arena = Arena(self.budget)
        self.n_slots = n_slots
        self.max_batch_frames = max_batch_frames
        self.clock = clock or time.perf_counter
        self.queue: List[Request] = []
        self.inflight: List[_InFlight] = []
        self.done: List[Request] = []
        self.out_bytes = 0
        self.peak_bytes = 0
        self.batches = 0
        self.batch_sizes: List[int] = []
        self.overlapped_launches = 0   # batches launched while another was in flight
        self.failed_batches = 0
        self.t0 = 0.0                  # engine-clock origin of arrival and finish times

    # ------------------------------------------------------------ accounting
    def bytes_in_use(self) -> int:
        return self.arena.bytes_in_use + self.out_bytes

    def _fits_alone(self, r: Request) -> bool:
        return self.ex.workspace_bytes([r.shape]) + self.ex.out_bytes(r.shape) <= self.budget

    # -------------------------------------------------------------- requests
    def submit(self, r: Request) -> None:
        if not r.shape or r.shape == (0, 0, 0):
            r.shape = self.ex.shape_of(r.image)
        if not self._fits_alone(r):
            r.rejected = True
            self.done.append(r)
            return
        self.queue.append(r)

    def _free_slot(self) -> Optional[int]:
        busy = {f.slot for f in self.inflight}
        for s in range(self.n_slots):
            if s not in busy:
                return s
        return None

    def poll(self) -> List[Request]:
        """Retire finished batches; returns the requests that finished."""
        finished: List[Request] = []
        still: List[_InFlight] = []
        now = self.clock() - self.t0
        for f in self.inflight:
            t = self.ex.finished_at(f.handle, now)
            if t is None:
                still.append(f)
                continue
            for r in f.requests:
                r.finished = t
                finished.append(r)
            self.ex.release(f.handle)
            self.arena.release(f.arena_off)
            self.out_bytes -= f.out_bytes
        self.inflight = still
        self.done.extend(finished)
        return finished

    def admit(self) -> int:
        """Launch batches while a slot is free and the queue head fits; returns
        the number of batches launched."""
        launched = 0
        while self.queue:
            slot = self._free_slot()
            if slot is None:
                break
            take: List[Request] = []
            need_ws = 0
            need_out = 0
            for r in self.queue:                       # FIFO prefix that fits
                if len(take) == self.max_batch_frames:
                    break
                ws = self.ex.workspace_bytes([q.shape for q in take] + [r.shape])
                ob = need_out + self.ex.out_bytes(r.shape)
                if _align(ws) + self.arena.bytes_in_use + self.out_bytes + ob > self.budget:
                    break
                take.append(r)
                need_ws, need_out = ws, ob
            if not take:
                break
            off = self.arena.alloc(need_ws)
            if off is None:                           # fragmented: wait for frees
                break
            now = self.clock() - self.t0
            for r in take:
                r.admitted = now
                r.batch_id = self.batches
            del self.queue[:len(take)]
            try:
                handle = self.ex.launch(take, slot, off, need_ws)
            except Exception as e:                    # this batch fails alone
                self.arena.release(off)
                for r in take:
                    r.failed = True
                    r.error = f"{type(e).__name__}: {e}"
                self.done.extend(take)
                self.failed_batches += 1
                continue
            if self.inflight:
                self.overlapped_launches += 1
            self.inflight.append(_InFlight(self.batches, slot, take, handle, off, _align(need_ws), need_out))
            self.out_bytes += need_out
            self.peak_bytes = max(self.peak_bytes, self.bytes_in_use())
            self.batches += 1
            self.batch_sizes.append(len(take))
            launched += 1
        return launched

    def idle(self) -> bool:
        return not self.queue and not self.inflight


def run(engine: Engine, requests: Sequence[Request], sleep: Callable[[float], None] = time.sleep,
        poll_interval: float = 50e-6) -> dict:
    """Feed requests at their arrival times (seconds after the start) and run
    the loop until every request has finished or been rejected."""
    pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
    t0 = engine.clock()
    engine.t0 = t0
    engine.ex.start(t0)
    i = 0
    while i < len(pending) or not engine.idle():
        now = engine.clock() - t0
        while i < len(pending) and pending[i].arrival <= now:
            engine.submit(pending[i])
            i += 1
        engine.poll()
        engine.admit()
        if i < len(pending) or not engine.idle():
            nxt = pending[i].arrival - (engine.clock() - t0) if i < len(pending) else poll_interval
            sleep(max(0.0, min(poll_interval, nxt)))
    return summarize(engine, requests, t0)


def summarize(engine: Engine, requests: Sequence[Request], t0: float) -> dict:
    ok = [r for r in requests if not r.rejected and not r.failed]
    lat = np.array([r.latency for r in ok], dtype=np.float64) * 1e3 if ok else np.zeros(0)
    span = (max(r.finished for r in ok) - min(r.arrival for r in ok)) if ok else 0.0
    return {
        "requests": len(requests),
        "completed": len(ok),
        "rejected": sum(1 for r in requests if r.rejected),
        "failed": sum(1 for r in requests if r.failed),
        "failed_batches": engine.failed_batches,
        "batches": engine.batches,
        "mean_batch_frames": float(np.mean(engine.batch_sizes)) if engine.batch_sizes else 0.0,
        "overlapped_launches": engine.overlapped_launches,
        "latency_ms": {"p50": float(np.percentile(lat, 50)) if len(lat) else None,
                       "p99": float(np.percentile(lat, 99)) if len(lat) else None,
                       "max": float(lat.max()) if len(lat) else None},
        "frames_per_s": len(ok) / span if span > 0 else None,
        "makespan_s": span,
        "peak_hbm_bytes": engine.peak_bytes,
        "budget_bytes": engine.budget,
    }


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate, from 0."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, n)
    return np.cumsum(gaps) - gaps[0]


# ---------------------------------------------------------------- executors
class FakeExecutor:
    """CPU stand-in: a batch takes `cost(shapes)` seconds after launch on its
    slot; memory sizes follow the real layout rules given as callables."""

    def __init__(self, clock: Callable[[], float], cost: Callable[[List[Tuple[int, int, int]]], float],
                 workspace_bytes: Callable[[List[Tuple[int, int, int]]], int]):
        self.clock = clock
        self.cost = cost
        self._ws = workspace_bytes
        self.launches: List[Tuple[int, List[int], float]] = []

    def start(self, t0):
        self.t0 = t0

    def shape_of(self, image):
        return tuple(image)

    def workspace_bytes(self, shapes):
        return self._ws(list(shapes))

    def out_bytes(self, shape):
        c, h, w = shape
        return _align(4 * c * h * w)

    def launch(self, reqs, slot, off, nbytes):
        now = self.clock()
        self.launches.append((slot, [r.rid for r in reqs], now))
        return {"end": now + self.cost([r.shape for r in reqs])}

    def finished_at(self, h, now):
        return h["end"] - self.t0 if self.clock() >= h["end"] else None

    def release(self, h):
        pass


class GpuExecutor:
    """Runs each admitted batch through p2s_batch_create/upload/launch on the
    slot's stream, inside the engine's arena (one device buffer of the budget,
    allocated once).  Every request brings its own output buffer (Request.out,
    the shape of its image), so the executor allocates nothing per batch; a
    batch is finished once the event recorded after its kernels has
    completed, at the engine-clock time of the poll that sees it."""

    def __init__(self, sim, precision: str, arena_bytes: int, n_slots: int, options: Optional[dict] = None):
        import torch
        self.torch = torch
        self.sim = sim
        self.precision = precision
        self.options = options or {}
        self.arena = torch.empty(_align(arena_bytes), dtype=torch.uint8, device="cuda")
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]

    def start(self, t0):
        self.torch.cuda.synchronize()

    def shape_of(self, image):
        return tuple(int(v) for v in image.shape)

    def workspace_bytes(self, shapes):
        from . import p2s
        return p2s.batch_workspace_bytes(list(shapes), self.sim.n_zernike, self.sim.basis.K, self.sim.corr_len_px)

    def out_bytes(self, shape):
        return 0                                      # outputs are the caller's

    def launch(self, reqs, slot, off, nbytes):
        from . import p2s
        torch = self.torch
        for r in reqs:
            if r.out is None or tuple(r.out.shape) != tuple(r.image.shape):
                raise ValueError(f"request {r.rid}: needs an output buffer of its image's shape")
        s = self.streams[slot]
        ws = self.arena[off: off + _align(nbytes)]
        b = p2s.Batch([r.image for r in reqs], [r.out for r in reqs], [r.d_over_r0 for r in reqs],
                      [r.seed for r in reqs], self.sim.basis, self.sim.net, self.precision, ws, self.sim.n_zernike,
                      self.sim.corr_len_px, self.sim.q_sampling, **self.options)
        try:
            b.upload(stream=s)
            b.launch(stream=s)
        except Exception:
            b.close()
            raise
        ev = torch.cuda.Event()
        ev.record(s)
        return (b, ev)

    def finished_at(self, h, now):
        b, ev = h
        return now if ev.query() else None

    def release(self, h):
        b, ev = h
        b.close()
