"""Autotuner for the tier thresholds and accumulator sizes of a product shape.

The tunable knobs are the fields of ``sg_tuning``: the tiny/mid flops
thresholds of the binning step, the LDS bytes and workgroup size of the mid
tier and of the heavy tier (mid capacity and heavy window width follow from
them), the number of persistent workgroups per compute unit and the budget
of per-window entry records (which pay off when the numeric phase is
replayed).
A search times whole steps (symbolic + numeric, or numeric only for a
structure-reusing caller) of the actual operands and keeps the fastest
setting; candidates the library rejects are skipped. Results are cached in a
JSON file under a shape-class key (semiring, output format, launch form and
log2 buckets of the total flops, largest vector flops and output vectors), so
products of the same class reuse the setting without searching again.

Every candidate computes the same output (the tiers are exact); the tuner
only changes where the work runs.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

from . import binding as B

# Coordinate-descent search space, most influential knob first.
SPACE: Dict[str, List[int]] = {
    "heavy_lds_bytes": [78848, 131072, 159744],
    "heavy_threads": [512, 1024],
    "lds_bytes": [32768, 49152, 65536, 78848, 98304, 131072, 161792],
    "blocks_per_cu": [1, 2, 3, 4],
    "block_threads": [256, 512],
    "mid_max_ub": [4096, 16384, 65535],
    "tiny_max_flops": [16, 32, 64],
    "entry_mb": [0, 1024],
    "small_max_flops": [0, 512, 1024],
}


def default_cache_path() -> str:
    return os.environ.get("SG_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sg_spgemm",
                                                        "tuning.json"))


def _b2(x: int) -> int:
    return int(math.floor(math.log2(x))) if x > 0 else -1


def shape_key(semiring: str, out_fmt: str, form: str, infos: Sequence[dict]) -> str:
    flops = sum(i["flops"] for i in infos)
    vmax = max((i["max_vec_flops"] for i in infos), default=0)
    nvec = sum(i["n_out_vec"] for i in infos)
    return f"{semiring}/{out_fmt}/{form}/p{_b2(len(infos))}/f{_b2(flops)}/v{_b2(vmax)}/n{_b2(nvec)}"


class TuneCache:
    """JSON map shape key -> {"tuning": {field: value}, "ms": best, "default_ms": ...}."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or default_cache_path()
        self.data: Dict[str, dict] = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    def get(self, key: str) -> Optional[dict]:
        return self.data.get(key)

    def put(self, key: str, entry: dict):
        self.data[key] = entry
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


class _Runner:
    """Times one candidate: `reps` steps after one warm-up, median wall time with a sync."""

    def __init__(self, semiring, As, Bs, group, ngroup, out_fmt, form, reps):
        import torch
        self.torch = torch
        self.args = (semiring, list(As), list(Bs), group, ngroup)
        self.out_fmt = out_fmt
        self.form = form
        self.reps = reps
        self.ws = None

    def plan(self, tuning):
        sr, As, Bs, group, ngroup = self.args
        p = B.spgemm_symbolic(sr, As, Bs, group, ngroup, out_fmt=self.out_fmt, tuning=tuning, ws=self.ws)
        self.ws = p.ws
        return p

    def time(self, tuning) -> float:
        torch = self.torch
        launch = B.spgemm_batched if self.form == "batched" else B.spgemm_numeric
        ts = []
        if self.form == "numeric_reuse":
            p = self.plan(tuning)
            outs = p.alloc_outputs()
            for r in range(self.reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                B.spgemm_batched(p, outs)
                torch.cuda.synchronize()
                if r:
                    ts.append(time.perf_counter() - t0)
            p.destroy()
        else:
            outs = None
            for r in range(self.reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                p = self.plan(tuning)
                if outs is None:
                    outs = p.alloc_outputs()
                launch(p, outs)
                torch.cuda.synchronize()
                if r:
                    ts.append(time.perf_counter() - t0)
                p.destroy()
        ts.sort()
        return ts[len(ts) // 2] * 1e3


# Joint settings for grouped plans that are replayed (a SUMMA share, a
# batch of Galerkin products): knobs that only pay off together, tried as
# whole candidates before the coordinate descent starts from the best one.
REPLAY_PRESETS: List[Dict[str, int]] = [
    {"entry_mb": 1024},
    {"entry_mb": 1024, "mid_max_ub": 2048},
    {"entry_mb": 1024, "mid_max_ub": 1024},
    {"entry_mb": 256},
    {"entry_mb": 1024, "heavy_lds_bytes": 159744, "heavy_threads": 1024, "lds_bytes": 159744, "block_threads": 1024},
]
REPLAY_SPACE: Dict[str, List[int]] = {
    "entry_mb": [0, 256, 1024],
    "small_max_flops": [0, 512, 1024],
    "mid_max_ub": [1024, 2048, 65535],
    "tiny_max_flops": [32, 64],
    "bitmap_mb": [0, 4096],
}


def autotune(semiring: str, As: Sequence, Bs: Sequence, group=None, ngroup=None, out_fmt: Optional[str] = None,
             form: str = "numeric", space: Optional[Dict[str, List[int]]] = None, reps: int = 3, sweeps: int = 1,
             cache: Optional[TuneCache] = None, force: bool = False, log=None,
             presets: Optional[Sequence[Dict[str, int]]] = None) -> dict:
    """Search ``space`` by coordinate descent from the default setting (or
    from the fastest of ``presets``, whole settings tried first).

    form: "numeric" (symbolic + per-tier launches), "batched" (symbolic + one
    persistent launch) or "numeric_reuse" (the persistent launch alone, as a
    graph replay would run it). Returns {"key", "tuning" (overrides),
    "ms", "default_ms", "tried"} and stores it in ``cache`` if given; a cached
    entry is returned as is unless ``force``.
    """
    out_fmt = out_fmt or As[0].fmt
    space = space or SPACE
    run = _Runner(semiring, As, Bs, group, ngroup, out_fmt, form, reps)
    p0 = run.plan(None)
    key = shape_key(semiring, out_fmt, form, p0.infos)
    p0.destroy()
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            return dict(hit, key=key, cached=True)
    best = {}
    best_ms = default_ms = run.time(None)
    tried = [({}, default_ms)]

    def attempt(cand):
        try:
            ms = run.time(B.make_tuning(semiring, **cand))
        except B.SgError as e:  # the library refused this setting for this shape
            if log:
                log(f"[autotune] {cand}: {e}")
            return None
        tried.append((cand, ms))
        if log:
            log(f"[autotune] {cand}: {ms:.3f} ms")
        return ms

    for cand in presets or []:
        ms = attempt(dict(cand))
        if ms is not None and ms < best_ms * 0.98:
            best, best_ms = dict(cand), ms
    for _ in range(sweeps):
        improved = False
        for field, values in space.items():
            for v in values:
                cand = dict(best, **{field: v})
                if cand == best:
                    continue
                ms = attempt(cand)
                if ms is None:
                    continue
                if ms < best_ms * 0.98:
                    best, best_ms, improved = cand, ms, True
        if not improved:
            break
    entry = {"tuning": best, "ms": best_ms, "default_ms": default_ms, "tried": len(tried)}
    if cache is not None:
        cache.put(key, entry)
    return dict(entry, key=key, cached=False)


def tuned(semiring: str, As: Sequence, Bs: Sequence, group=None, ngroup=None, out_fmt: Optional[str] = None,
          form: str = "numeric", cache: Optional[TuneCache] = None):
    """The cached tuning for this product's shape class (None: use the defaults)."""
    cache = cache or TuneCache()
    out_fmt = out_fmt or As[0].fmt
    p0 = B.spgemm_symbolic(semiring, list(As), list(Bs), group, ngroup, out_fmt=out_fmt)
    key = shape_key(semiring, out_fmt, form, p0.infos)
    p0.destroy()
    hit = cache.get(key)
    return None if hit is None else B.make_tuning(semiring, **hit["tuning"])
