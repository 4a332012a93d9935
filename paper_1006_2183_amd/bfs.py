"""Masked multi-level breadth-first search on the device, and its served form.

Multi-source BFS is a sequence of sparse products (paper, Section 6.2.2):
with A the n x n adjacency matrix held column-major (A(i, k): an edge from
k to i) and X_0 the n x k frontier with source s_c in column c, level d + 1
is X_{d+1} = (A X_d) restricted to the positions not yet visited, and the
visited set grows by X_{d+1}. Every column is an independent search; the
visited sets are one bitmap per column (n bits), passed to the product as a
complement mask, so a reached vertex is never produced again and the
frontier never needs a separate filtering pass. All steps run in the HIP
library: the first frontier is built from the sources on the device
(sg_coo_compress / sg_coo_emit), each level is one masked product
(sg_spgemm_symbolic_masked, then the persistent numeric launch), and the
visited bitmaps are updated on the device (sg_mask_set).

``BfsServer`` serves BFS requests with iteration-level continuous batching:
every iteration multiplies the current frontiers of ALL active requests in
one grouped, masked product (one group per request, each at its own depth:
the "level mix"), so requests that arrive while others are in flight join at
the next iteration instead of waiting for the earlier searches to finish.
Admission is by the visited-bitmap memory a request needs (its columns times
ceil(n / 32) words) against a pool, and by a cap on active requests.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import binding as B


_staging = None


def sources_frontier(sources, n: int, stream=None):
    """X_0: the n x k boolean frontier with sources[c] in column c, built on the device
    from one host-to-device copy of its triples."""
    import torch
    from .serve import PinnedStaging
    global _staging
    if _staging is None:
        _staging = PinnedStaging()
    src = np.asarray(sources, dtype=np.int32)
    k = int(src.size)
    st = stream if stream is not None else torch.cuda.current_stream()
    dev = _staging.to_device(np.concatenate([src, np.arange(k, dtype=np.int32)]), "cuda", st)
    return B.coo_to_sparse("or_and_bool", dev[:k], dev[k:], None, n, k, "csc", stream=stream)


class MaskedBFS:
    """Level-synchronous multi-source BFS of one request on a resident A."""

    def __init__(self, A, tuning=None):
        if A.fmt != "csc" or A.nrows != A.ncols:
            raise ValueError("a square column-major (csc) adjacency matrix is expected")
        self.A, self.tuning = A, tuning

    def run(self, sources, max_levels: Optional[int] = None, stream=None) -> List:
        """Frontiers X_0, X_1, ... (device CSC n x k, level d = the vertices first
        reached at depth d per column), until every column's frontier is empty
        or max_levels levels beyond the sources are done."""
        n = self.A.nrows
        X = sources_frontier(sources, n, stream)
        visited = B.Mask.zeros(X.ncols, n, complement=True)
        B.mask_set([X], [visited], stream)
        levels = [X]
        while max_levels is None or len(levels) <= max_levels:
            plan = B.spgemm_symbolic("or_and_bool", [self.A], [X], out_fmt="csc", tuning=self.tuning, stream=stream,
                                     masks=[visited])
            if plan.infos[0]["nnz"] == 0:
                plan.destroy()
                break
            (Y,) = plan.alloc_outputs()
            B.spgemm_batched(plan, [Y], stream)
            plan.destroy()
            B.mask_set([Y], [visited], stream)
            levels.append(Y)
            X = Y
        return levels


@dataclasses.dataclass
class BfsRequest:
    rid: int
    arrival: float
    sources: np.ndarray
    max_levels: int
    status: str = "queued"
    start: float = float("nan")
    done: float = float("nan")
    levels: list = dataclasses.field(default_factory=list)
    # device state while active
    X: object = None
    visited: object = None


class BfsServer:
    """Iteration-level continuous batching of BFS requests (see the module text).

    batched=False gives the FIFO baseline: one request at a time, each level
    its own plain product, in arrival order."""

    def __init__(self, A, pool_bytes: int = 8 << 30, max_active: int = 64, batched: bool = True, tuning=None,
                 clock: Callable[[], float] = time.perf_counter):
        import torch
        self.torch = torch
        self.A, self.tuning = A, tuning
        self.n = A.nrows
        self.words = (self.n + 31) // 32
        self.pool = int(pool_bytes)
        self.free = int(pool_bytes)
        self.max_active = max_active if batched else 1
        self.batched = batched
        self.clock = clock
        self.iterations = 0
        self.mix: List[Dict[int, int]] = []  # per iteration: depth -> active requests at that depth

    def _bytes(self, r: BfsRequest) -> int:
        return len(r.sources) * self.words * 4

    def _start(self, r: BfsRequest, now: float):
        r.status, r.start = "running", now
        r.X = sources_frontier(r.sources, self.n)
        r.visited = B.Mask.zeros(r.X.ncols, self.n, complement=True)
        B.mask_set([r.X], [r.visited])
        r.levels = [r.X]

    def _finish(self, r: BfsRequest, t: float):
        r.status, r.done = "done", t
        r.X = None
        r.visited = None  # the bitmap memory returns to the pool
        self.free += self._bytes(r)

    def _iterate(self, active: List[BfsRequest]):
        """One masked product for every active request's current frontier."""
        n = len(active)
        self.mix.append({d: sum(1 for r in active if len(r.levels) - 1 == d) for d in
                         sorted(set(len(r.levels) - 1 for r in active))})
        plan = B.spgemm_symbolic("or_and_bool", [self.A] * n, [r.X for r in active], list(range(n)), n,
                                 out_fmt="csc", tuning=self.tuning, masks=[r.visited for r in active])
        Ys = plan.alloc_outputs()
        B.spgemm_batched(plan, Ys)
        infos = plan.infos
        plan.destroy()
        B.mask_set(Ys, [r.visited for r in active])
        self.iterations += 1
        ended = []
        for r, Y, info in zip(active, Ys, infos):
            if info["nnz"] == 0:
                ended.append(r)
                continue
            r.levels.append(Y)
            r.X = Y
            if len(r.levels) - 1 >= r.max_levels:
                ended.append(r)
        return ended

    def run(self, requests: Sequence[BfsRequest]) -> List[BfsRequest]:
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: List[BfsRequest] = []
        active: List[BfsRequest] = []
        finished: List[BfsRequest] = []
        t0 = self.clock()
        i = 0
        while i < len(pending) or waiting or active:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                waiting.append(pending[i])
                i += 1
            # admission: arrival order, by visited-bitmap memory and the active cap
            while waiting and len(active) < self.max_active:
                r = waiting[0]
                need = self._bytes(r)
                if need > self.pool:
                    waiting.pop(0)
                    r.status, r.done = "rejected", now
                    finished.append(r)
                    continue
                if need > self.free:
                    break
                waiting.pop(0)
                self.free -= need
                self._start(r, now)
                if r.max_levels <= 0:
                    self.torch.cuda.current_stream().synchronize()
                    self._finish(r, self.clock() - t0)
                    finished.append(r)
                    continue
                active.append(r)
            if not active:
                continue
            ended = self._iterate(active)
            if ended:
                # results complete once the iteration's launches have run
                self.torch.cuda.current_stream().synchronize()
                t = self.clock() - t0
                for r in ended:
                    self._finish(r, t)
                    finished.append(r)
                active = [r for r in active if r not in ended]
        return finished


def bfs_latency(reqs: Sequence[BfsRequest]) -> Dict[str, float]:
    done = [r for r in reqs if r.status == "done"]
    lat = np.array([r.done - r.arrival for r in done]) if done else np.zeros(0)
    span = (max(r.done for r in done) - min(r.arrival for r in done)) if done else 0.0
    return {"done": len(done), "rejected": sum(r.status == "rejected" for r in reqs),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else float("nan"),
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else float("nan"),
            "mean_ms": float(lat.mean() * 1e3) if lat.size else float("nan"),
            "throughput_rps": len(done) / span if span > 0 else float("nan")}
