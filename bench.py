#!/usr/bin/env python3
"""Benchmark of the plain local product C = A A on one MI355X.

Workload: A is an R-MAT matrix of scale 18 (n = 262,144) and edge factor 16
with quadrant probabilities (0.57, 0.19, 0.19, 0.05), duplicates summed,
FP64 values uniform(0, 1), in CSR; the (+,*) semiring. One step is one pass
of the whole plain path on device-resident operands: symbolic phase (flops
per row, tier binning, exact row counts, output pointers; it ends with one
host synchronisation to learn the output size) and the numeric phase into
an exactly sized output. The value is useful multiplications per second
(flops of C = A A divided by the step time), in G/s.

The JSON line also carries the roofline of the dominant numeric kernel
(algorithmic HBM bytes of the vectors it processes divided by its launch
time, measured with HIP events recorded by the library on the launch
stream), the same run under (min,+) int32, and the CPU oracle's rate on a
bounded row sample of the same product (the oracle is the test reference,
run here only to report a CPU baseline).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "semiring GFLOP/s (useful mul-adds) + HBM % of peak; batched vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0
RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)
VALUE_BYTES = {"plus_times_f64": 8, "plus_times_f32": 4, "min_plus_i32": 4, "or_and_bool": 0}
DTYPE = {"plus_times_f64": "f64", "plus_times_f32": "f32", "min_plus_i32": "i32", "or_and_bool": "bool"}
TIER_NAMES = ("tiny", "mid", "heavy")
KERNEL_NAMES = {"heavy": "k_heavy", "mid": "k_mid", "tiny": "k_tiny"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1006_2183_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(info, tier, s):
    """Algorithmic HBM bytes of the numeric work of one tier.

    Stream the tier's vectors of the streamed operand ((4 + s) per stored
    entry, 8 per vector pointer), read the pointer pair of every referenced
    gathered vector (16 per stored entry), gather the referenced entries
    ((4 + s) per multiplication), and write the output ((4 + s) per entry
    and 8 per vector pointer).
    """
    x = TIER_NAMES.index(tier)
    nvec = {"tiny": info["n_tiny"], "mid": info["n_mid"], "heavy": info["n_heavy"]}[tier]
    sent = info["tier_sent"][x]
    flops = info["tier_flops"][x]
    nnz = info["tier_nnz"][x]
    return (4 + s) * sent + 8 * (nvec + 1) + 16 * sent + (4 + s) * flops + (4 + s) * nnz + 8 * (nvec + 1)


def load_traffic(kernel, workload, semiring):
    """Measured HBM bytes per launch from the committed counter summary, if still current."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(f"{workload}/{semiring}/{kernel}")
        if not e or e.get("kernel_hash") != kernel_source_hash():
            return None
        return e.get("bytes_per_launch")
    except Exception:
        return None


def run_product(sg, torch, semiring, A, steps, warmup, tuning):
    """Time `steps` full plain products; returns timings and the plan info."""
    dA = sg.DevMat.from_host(A, "cuda", semiring)
    ws = None
    C = None
    info = None

    def step(profile):
        nonlocal ws, C, info
        plan = sg.spgemm_symbolic(semiring, [dA], [dA], tuning=tuning, ws=ws)
        ws = plan.ws
        info = plan.infos[0]
        if C is None:
            C = plan.alloc_outputs()
        if profile:
            plan.profile(True)
        sg.spgemm_numeric(plan, C)
        kt = plan.kernel_times() if profile else None
        plan.destroy()
        return kt

    for _ in range(warmup):
        step(True)
    torch.cuda.synchronize()
    times = {k: [] for k in ("heavy", "mid", "tiny", "ptr")}
    t0 = time.perf_counter()
    for _ in range(steps):
        kt = step(True)
        for k in times:
            times[k].append(kt[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # symbolic alone (host clock around the call, which ends in a sync)
    sym = []
    for _ in range(max(1, min(steps, 3))):
        ts = time.perf_counter()
        plan = sg.spgemm_symbolic(semiring, [dA], [dA], tuning=tuning, ws=ws)
        sym.append(time.perf_counter() - ts)
        plan.destroy()
    del C
    return {
        "ms_per_step": (t1 - t0) * 1e3 / steps,
        "kernel_ms": {k: float(np.mean(v)) for k, v in times.items()},
        "symbolic_ms": float(np.median(sym)) * 1e3,
        "info": info,
    }


def rows_subset(A, rows):
    import types
    lens = np.diff(A.ptr)[rows]
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=ptr[1:])
    sel = np.concatenate([np.arange(A.ptr[r], A.ptr[r + 1]) for r in rows])
    return types.SimpleNamespace(fmt="csr", nrows=len(rows), ncols=A.ncols, ptr=ptr, idx=A.idx[sel],
                                 val=None if A.val is None else A.val[sel], vid=None)


def cpu_baseline(semiring, A, total_flops, seconds):
    """The oracle, single-threaded, on a uniform random row sample of C = A A."""
    import oracle
    rng = np.random.default_rng(7)
    n = A.nrows
    # calibrate on a small sample, then size the sample for about `seconds`
    probe = np.sort(rng.choice(n, max(64, n // 2000), replace=False))
    t = time.perf_counter()
    _, f0 = oracle.spgemm(semiring, rows_subset(A, probe), A)
    dt = max(time.perf_counter() - t, 1e-3)
    rate = f0 / dt
    frac = min(1.0, seconds * rate / max(total_flops, 1))
    k = max(64, int(round(frac * n)))
    rows = np.sort(rng.choice(n, k, replace=False))
    t = time.perf_counter()
    _, fl = oracle.spgemm(semiring, rows_subset(A, rows), A)
    dt = time.perf_counter() - t
    return {
        "value": fl / dt / 1e9,
        "unit": "GFLOP/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"C(R,:) = A(R,:) A for {k} of {n} rows drawn uniformly (seed 7): {fl} multiplications in "
                  f"{dt:.1f} s, single-threaded C Gustavson with a dense accumulator",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=18)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--semiring", default="plus_times_f64")
    ap.add_argument("--no-i32", action="store_true", help="skip the (min,+) int32 run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tuning", default=None, help="JSON object of sg_tuning overrides")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="run only a device copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU's share; the build targets a single "
                                   "MI355X and runs no collectives, so --gpus must be 1"}), flush=True)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8}), flush=True)
        return

    import paper_1006_2183_amd as sg
    import workloads as W
    sg.load_library()

    tune_kw = json.loads(args.tuning) if args.tuning else {}
    workload = f"rmat_s{args.scale}_ef{args.edge_factor}_AxA_plain"
    results = {}
    semirings = [args.semiring] + ([] if args.no_i32 or args.semiring == "min_plus_i32" else ["min_plus_i32"])
    A_main = None
    for sr in semirings:
        log(f"[bench] generating R-MAT scale {args.scale} ef {args.edge_factor} ({sr})")
        A = W.rmat_matrix(args.scale, args.edge_factor, sr, "csr", seed=args.seed, abcd=RMAT_ABCD)
        if sr == args.semiring:
            A_main = A
        tuning = sg.make_tuning(sr, **tune_kw) if tune_kw else None
        log(f"[bench] {sr}: nnz(A) = {A.nnz}; warmup {args.warmup}, steps {args.steps}")
        r = run_product(sg, torch, sr, A, args.steps, args.warmup, tuning)
        info = r["info"]
        r["gflops"] = info["flops"] / (r["ms_per_step"] / 1e3) / 1e9
        log(f"[bench] {sr}: {r['ms_per_step']:.2f} ms/step, {r['gflops']:.1f} G mul-add/s, "
            f"kernels {r['kernel_ms']}, symbolic {r['symbolic_ms']:.2f} ms")
        results[sr] = (A, r)

    A, r = results[args.semiring]
    info = r["info"]
    s = VALUE_BYTES[args.semiring]
    km = r["kernel_ms"]
    dom = max(("heavy", "mid", "tiny"), key=lambda k: km[k])
    algo = algorithmic_bytes(info, dom, s)
    achieved = algo / (km[dom] / 1e3) / 1e9 if km[dom] > 0 else 0.0
    roofline = {
        "bound": "hbm",
        "kernel": KERNEL_NAMES[dom],
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": load_traffic(KERNEL_NAMES[dom], workload, args.semiring),
        "algorithmic_bytes_per_launch": int(algo),
        "launch_ms": round(km[dom], 4),
    }
    numeric_ms = km["heavy"] + km["mid"] + km["tiny"] + km["ptr"]
    numeric_algo = sum(algorithmic_bytes(info, t, s) for t in TIER_NAMES)
    out = {
        "metric": METRIC,
        "value": round(r["gflops"], 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.semiring],
        "data": "synthetic",
        "config": {
            "workload": workload,
            "semiring": args.semiring,
            "format": "csr",
            "n": A.nrows,
            "nnz_A": A.nnz,
            "flops": info["flops"],
            "nnz_C": info["nnz"],
            "rmat_abcd": list(RMAT_ABCD),
            "seed": args.seed,
            "tuning": sg.make_tuning(args.semiring, **tune_kw).as_dict(),
        },
        "roofline": roofline,
        "phases_ms": {
            "symbolic": round(r["symbolic_ms"], 3),
            "numeric_kernels": round(numeric_ms, 3),
            "heavy": round(km["heavy"], 3), "mid": round(km["mid"], 3), "tiny": round(km["tiny"], 3),
            "pointers": round(km["ptr"], 3),
        },
        "numeric_phase_hbm": {
            "algorithmic_bytes": int(numeric_algo),
            "achieved_GBs": round(numeric_algo / (numeric_ms / 1e3) / 1e9, 1) if numeric_ms > 0 else None,
        },
        "tiers": {t: {"vectors": info[f"n_{t}"], "flops": info["tier_flops"][i], "nnz": info["tier_nnz"][i]}
                  for i, t in enumerate(TIER_NAMES)},
    }
    if "min_plus_i32" in results and args.semiring != "min_plus_i32":
        _, ri = results["min_plus_i32"]
        out["min_plus_i32"] = {"value": round(ri["gflops"], 3), "unit": "GFLOP/s",
                               "ms_per_step": round(ri["ms_per_step"], 4),
                               "kernel_ms": {k: round(v, 3) for k, v in ri["kernel_ms"].items()}}
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a row sample")
        out["cpu_baseline"] = cpu_baseline(args.semiring, A_main, info["flops"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
