"""Serving loop: continuous batching of sparse products against a resident operand.

Requests are products Y_r = A (x) X_r with A resident on the device (the
multi-source breadth-first expansion of Section 6.2.2: A is the adjacency
matrix, X_r a tall-skinny frontier, (or, and) semiring). The loop

* admits a waiting request when a batch slot is free and its output-size
  bound (the symbolic bound: sum over the stored entries (k, s) of X_r of
  nnz(A(:, k)), which is also its flops) fits in the free part of the output
  memory pool; a request whose bound exceeds the whole pool is rejected, and
  one that waited past its deadline is cancelled before launch;
* plans every admitted batch as one grouped product (one output per request)
  and runs it as one persistent launch on one of several streams, so the
  next batch is planned and launched while earlier ones compute
  (continuous batching; beside a batch already in flight, once at least
  two requests wait);
* completes requests when their batch's event has fired, frees their pool
  bytes and records latency (completion - arrival).

``FifoExecutor`` runs one request per launch in arrival order, the baseline.
``FrontierBatchExecutor`` / ``FrontierFifoExecutor`` take requests as they
arrive from a client (host triples of the frontier) and build the sparse
operand on the device. The scheduler is host-only logic; executors do the
device work.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds since the start of the run
    X: object                      # the right operand (executor-specific)
    ub: int                        # output-size bound (entries)
    deadline: Optional[float] = None
    status: str = "queued"         # queued, running, done, rejected, cancelled
    start: float = float("nan")
    done: float = float("nan")
    result: object = None


class Scheduler:
    """Admission and continuous batching, independent of the device.

    executor.launch(batch) -> handle; executor.poll(handle) -> bool (done);
    executor.finish(handle) -> list of results aligned with the batch.
    pool_entries: output entries that may be in flight at once.
    """

    def __init__(self, executor, pool_entries: int, max_batch: int = 64, max_inflight: int = 2,
                 clock: Callable[[], float] = time.perf_counter, idle: Callable[[], None] = lambda: None,
                 overlap_min_waiting: int = 2):
        self.ex = executor
        self.pool = int(pool_entries)
        self.free = int(pool_entries)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        # a batch is launched beside one already in flight only when at least
        # this many requests wait (1: whenever a slot is free). With 2, a lone
        # request waits for the batch on the device rather than slowing it
        # down (measured on served frontiers: p50 and p99 at 2000 requests/s
        # 10 to 30% lower than with 1, the same at 500 and 8000)
        self.overlap_min_waiting = overlap_min_waiting
        self.clock = clock
        self.idle = idle
        self.waiting: collections.deque = collections.deque()
        self.inflight: List = []
        self.finished: List[Request] = []
        self.batches = 0

    def _admit(self, now: float) -> List[Request]:
        batch = []
        while self.waiting and len(batch) < self.max_batch:
            r = self.waiting[0]
            if r.deadline is not None and now > r.deadline:
                self.waiting.popleft()
                r.status = "cancelled"
                r.done = now
                self.finished.append(r)
                continue
            if r.ub > self.pool:
                self.waiting.popleft()
                r.status = "rejected"
                r.done = now
                self.finished.append(r)
                continue
            if r.ub > self.free:
                break  # keep arrival order: wait for memory to free up
            self.waiting.popleft()
            self.free -= r.ub
            r.status = "running"
            r.start = now
            batch.append(r)
        return batch

    def _complete(self, now: float):
        keep = []
        for handle, batch in self.inflight:
            if self.ex.poll(handle):
                results = self.ex.finish(handle)
                t = self.clock() - self._t0
                for r, res in zip(batch, results):
                    r.result = res
                    r.status = "done"
                    r.done = t
                    self.free += r.ub
                    self.finished.append(r)
            else:
                keep.append((handle, batch))
        self.inflight = keep

    def run(self, requests: Sequence[Request]) -> List[Request]:
        """Serve requests whose `arrival` times follow the clock; returns them finished."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        self._t0 = self.clock()
        while pending or self.waiting or self.inflight:
            now = self.clock() - self._t0
            while pending and pending[0].arrival <= now:
                self.waiting.append(pending.popleft())
            if self.inflight:
                self._complete(now)
            launched = False
            if self.waiting and len(self.inflight) < self.max_inflight and (
                    not self.inflight or len(self.waiting) >= self.overlap_min_waiting):
                if hasattr(self.ex, "between"):
                    # the executor calls back between the host-blocking steps of
                    # a launch, so batches already in flight are retired (and
                    # their completion times taken) while the next one is planned
                    self.ex.between = lambda: self._complete(self.clock() - self._t0) if self.inflight else None
                batch = self._admit(self.clock() - self._t0)
                if batch:
                    # launch first: its callbacks may replace self.inflight
                    handle = self.ex.launch(batch)
                    self.inflight.append((handle, batch))
                    self.batches += 1
                    launched = True
            if not launched:
                self.idle()
        return self.finished


def latency_stats(reqs: Sequence[Request]) -> Dict[str, float]:
    done = [r for r in reqs if r.status == "done"]
    lat = np.array([r.done - r.arrival for r in done]) if done else np.zeros(0)
    span = (max(r.done for r in done) - min(r.arrival for r in done)) if done else 0.0
    return {
        "done": len(done),
        "rejected": sum(r.status == "rejected" for r in reqs),
        "cancelled": sum(r.status == "cancelled" for r in reqs),
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else float("nan"),
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else float("nan"),
        "mean_ms": float(lat.mean() * 1e3) if lat.size else float("nan"),
        "throughput_rps": len(done) / span if span > 0 else float("nan"),
    }


# ---------------------------------------------------------------------------
class PinnedStaging:
    """A reusable pinned host buffer for host-to-device copies on one stream: grown
    (allocated) only when a larger copy comes; before it is overwritten, the host
    waits for the event of the previous copy (normally long complete), so copies
    never read a buffer the host is rewriting. No per-copy pinned allocation, whose
    release could synchronise the device."""

    def __init__(self):
        self.buf = None
        self.done = None

    def to_device(self, arr: np.ndarray, device, stream):
        import torch
        if self.done is not None:
            self.done.synchronize()
        n = arr.size
        if self.buf is None or self.buf.numel() < n:
            self.buf = torch.empty(max(n, 1024), dtype=torch.int32, pin_memory=True)
        self.buf[:n].numpy()[:] = arr
        with torch.cuda.stream(stream):
            dev = self.buf[:n].to(device, non_blocking=True)
            self.done = torch.cuda.Event()
            self.done.record(stream)
        return dev


class GpuBatchExecutor:
    """Each batch is one grouped product: C_r = A (x) X_r for every request r of
    the batch, planned together and run as one persistent launch on one of
    `nstreams` streams (round robin). Request operands must be complete on the
    device when submitted; the executor synchronises once when it is created,
    and never makes its streams wait on the caller's stream per batch (on ROCm
    an event of the legacy default stream waits for every stream's work, which
    would serialise the batches)."""

    def __init__(self, semiring: str, A, out_fmt: Optional[str] = None, tuning=None, nstreams: int = 2,
                 timing: bool = False):
        import torch
        from . import binding as B
        self.B = B
        self.torch = torch
        self.semiring = semiring
        self.A = A
        self.out_fmt = out_fmt or A.fmt
        self.tuning = tuning
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.next = 0
        self.timing = timing
        self.intervals = []  # with timing: (stream index, start event, end event) per batch
        torch.cuda.synchronize()

    def launch(self, batch: Sequence[Request]):
        torch = self.torch
        si = self.next % len(self.streams)
        s = self.streams[si]
        self.next += 1
        n = len(batch)
        with torch.cuda.stream(s):
            if self.timing:
                t0 = torch.cuda.Event(enable_timing=True)
                t0.record(s)
            plan = self.B.spgemm_symbolic(self.semiring, [self.A] * n, [r.X for r in batch], list(range(n)), n,
                                          out_fmt=self.out_fmt, tuning=self.tuning, stream=s)
            outs = plan.alloc_outputs(self.A.ptr.device)
            self.B.spgemm_batched(plan, outs, s)
            ev = torch.cuda.Event(enable_timing=self.timing)
            ev.record(s)
            if self.timing:
                self.intervals.append((si, t0, ev))
        # the handle is released at once (host only); the workspace tensor and the
        # outputs stay referenced by the handle until the batch completes
        plan.destroy()
        return (ev, plan, outs)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle):
        ev, plan, outs = handle
        return outs


class FifoExecutor:
    """Baseline: one request per plain product, completed before the next starts."""

    def __init__(self, semiring: str, A, out_fmt: Optional[str] = None, tuning=None):
        import torch
        from . import binding as B
        self.B = B
        self.torch = torch
        self.semiring = semiring
        self.A = A
        self.out_fmt = out_fmt or A.fmt
        self.tuning = tuning

    def launch(self, batch: Sequence[Request]):
        outs = [self.B.spgemm(self.semiring, self.A, r.X, out_fmt=self.out_fmt, tuning=self.tuning) for r in batch]
        self.torch.cuda.synchronize()
        return outs

    def poll(self, handle) -> bool:
        return True

    def finish(self, handle):
        return handle


@dataclasses.dataclass
class Frontier:
    """A request's right operand as it arrives from the client: the n x k frontier
    as host triples (row ids, column ids in [0, k)); pattern only. The servers
    below build the compressed operand on the device from these."""
    rows: np.ndarray
    cols: np.ndarray
    k: int

    @classmethod
    def sources(cls, src) -> "Frontier":
        """One source per column (a breadth-first search's first frontier)."""
        src = np.asarray(src, dtype=np.int32)
        return cls(src, np.arange(src.size, dtype=np.int32), int(src.size))


class ColumnSlice:
    """Columns [c0, c1) of a column-major device result: one request's share of a
    batched product. ``to_host`` returns them as an n x (c1 - c0) CSC matrix."""

    def __init__(self, Y, c0: int, c1: int):
        self.Y, self.c0, self.c1 = Y, int(c0), int(c1)

    def to_host(self):
        import types
        ptr = self.Y.ptr[self.c0:self.c1 + 1].cpu().numpy()
        a, b = int(ptr[0]), int(ptr[-1])
        idx = self.Y.idx[a:b].cpu().numpy()
        val = None if self.Y.val is None else self.Y.val[a:b].cpu().numpy()
        return types.SimpleNamespace(fmt="csc", nrows=self.Y.nrows, ncols=self.c1 - self.c0, ptr=ptr - a, idx=idx,
                                     val=val, vid=None)


class FrontierBatchExecutor:
    """Continuous batching of frontier requests Y_r = A X_r ((or, and)) against a
    resident column-major A. A batch's frontiers are concatenated column-wise into
    one triple list (one host-to-device copy), compressed ON THE DEVICE into one
    CSC operand X = [X_1 | X_2 | ...] (sg_coo_compress / sg_coo_emit), and
    multiplied in ONE product Y = A X (symbolic, then the persistent launch) on one
    of `nstreams` streams; request r receives its columns of Y. The next batch is
    planned on the other stream while this one computes."""

    def __init__(self, A, nstreams: int = 2, tuning=None, timing: bool = False):
        import torch
        from . import binding as B
        self.B, self.torch, self.A, self.tuning = B, torch, A, tuning
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.staging = [PinnedStaging() for _ in range(nstreams)]
        self.next = 0
        self.timing = timing
        self.intervals = []
        self.between = None  # called between a launch's host-blocking steps (set by the scheduler)
        torch.cuda.synchronize()

    def _build(self, fronts, s, si=0):
        torch = self.torch
        ks = [f.k for f in fronts]
        off = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
        rows = np.concatenate([f.rows for f in fronts]).astype(np.int32)
        cols = np.concatenate([f.cols.astype(np.int64) + off[i] for i, f in enumerate(fronts)]).astype(np.int32)
        dev = self.staging[si].to_device(np.concatenate([rows, cols]), self.A.ptr.device, s)  # one copy on s
        n = rows.size
        X = self.B.coo_to_sparse("or_and_bool", dev[:n], dev[n:], None, self.A.nrows, int(off[-1]), "csc", stream=s)
        return X, off

    def launch(self, batch: Sequence[Request]):
        torch = self.torch
        si = self.next % len(self.streams)
        s = self.streams[si]
        self.next += 1
        with torch.cuda.stream(s):
                if self.timing:
                    t0 = torch.cuda.Event(enable_timing=True)
                    t0.record(s)
                X, off = self._build([r.X for r in batch], s, si)
                if self.between is not None:
                    self.between()
                plan = self.B.spgemm_symbolic("or_and_bool", [self.A], [X], out_fmt="csc", tuning=self.tuning,
                                              stream=s)
                if self.between is not None:
                    self.between()
                (Y,) = plan.alloc_outputs(self.A.ptr.device)
                self.B.spgemm_batched(plan, [Y], s)
                ev = torch.cuda.Event(enable_timing=self.timing)
                ev.record(s)
                if self.timing:
                    self.intervals.append((si, t0, ev))
        plan.destroy()  # host only; X, Y and the workspace stay referenced until completion
        return (ev, [ColumnSlice(Y, off[i], off[i + 1]) for i in range(len(batch))], (X, plan))

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle):
        return handle[1]


class FrontierFifoExecutor(FrontierBatchExecutor):
    """Baseline: one request per plain product (device-built operand, symbolic,
    per-tier numeric launches), completed before the next one starts."""

    def __init__(self, A, tuning=None):
        super().__init__(A, nstreams=1, tuning=tuning)

    def launch(self, batch: Sequence[Request]):
        # the end of the launch is polled, as the batched server polls its
        # events, so the two differ only in batching and overlap, not in how
        # a finished launch is noticed
        out = []
        s = self.torch.cuda.current_stream()
        for r in batch:
            X, _ = self._build([r.X], s)
            Y = self.B.spgemm("or_and_bool", self.A, X, out_fmt="csc", stream=s)
            out.append(ColumnSlice(Y, 0, r.X.k))
        ev = self.torch.cuda.Event()
        ev.record(s)
        while not ev.query():
            pass
        return out

    def poll(self, handle) -> bool:
        return True

    def finish(self, handle):
        return handle


def frontier_bound(colcount: np.ndarray, X) -> int:
    """Symbolic output bound of A X from a host copy of A's column counts:
    sum over the stored entries (k, s) of X of nnz(A(:, k)) (X a matrix or a
    Frontier)."""
    rows = X.rows if isinstance(X, Frontier) else X.idx
    return int(colcount[np.asarray(rows, dtype=np.int64)].sum())
