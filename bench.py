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


def host_info():
    """The host the oracle runs on: CPU model, logical CPUs, and the threads the
    all-core oracle uses (the CPUs this process may run on, at most 16: the GPU
    box's CPU share per GPU)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail, "threads": max(1, min(16, avail))}


def _oracle_timed(fn, threads):
    t = time.perf_counter()
    _, fl = fn(threads)
    return fl, time.perf_counter() - t


def cpu_baseline(semiring, A, total_flops, seconds):
    """The oracle on a uniform random row sample of C = A A: single-threaded, and on
    every available host core (row slices on a thread pool, each the same C routine)."""
    import oracle
    hi = host_info()
    rng = np.random.default_rng(7)
    n = A.nrows
    # calibrate single-threaded on a small sample, then size the sample so that the
    # single-threaded run takes about half of `seconds`
    probe = np.sort(rng.choice(n, max(64, n // 2000), replace=False))
    f0, dt = _oracle_timed(lambda th: oracle.spgemm(semiring, rows_subset(A, probe), A), 1)
    rate = f0 / max(dt, 1e-3)
    frac = min(1.0, 0.5 * seconds * rate / max(total_flops, 1))
    k = max(64, int(round(frac * n)))
    rows = np.sort(rng.choice(n, k, replace=False))
    sub = rows_subset(A, rows)
    fl1, dt1 = _oracle_timed(lambda th: oracle.spgemm(semiring, sub, A), 1)
    fln, dtn = _oracle_timed(lambda th: oracle.spgemm_threads(semiring, sub, A, threads=th), hi["threads"])
    return {
        "value": fln / dtn / 1e9,
        "unit": "GFLOP/s",
        "cores": hi["threads"],
        "kind": "oracle",
        "single_thread_value": fl1 / dt1 / 1e9,
        "host": hi,
        "sample": f"C(R,:) = A(R,:) A for {k} of {n} rows drawn uniformly (seed 7): {fl1} multiplications; "
                  f"single-threaded C Gustavson with a dense accumulator {dt1:.1f} s, on {hi['threads']} threads "
                  f"(row slices, same routine) {dtn:.1f} s",
    }


def cpu_rate(fn_by_threads, what):
    """Oracle rate of one bounded sample, single-threaded and on every available core."""
    hi = host_info()
    fl1, dt1 = _oracle_timed(fn_by_threads, 1)
    fln, dtn = _oracle_timed(fn_by_threads, hi["threads"])
    return {"value": round(fln / dtn / 1e9, 4), "unit": "GFLOP/s", "cores": hi["threads"], "kind": "oracle",
            "single_thread_value": round(fl1 / dt1 / 1e9, 4), "sample": what,
            "seconds": {"single_thread": round(dt1, 2), "all_cores": round(dtn, 2)}}


# ---------------------------------------------------------------------------
# Batched and served forms (reported beside the main line)

def _median_ms(torch, fn, reps):
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def _tier_bytes(infos, s):
    """Algorithmic numeric bytes summed over the tiers of every output of a plan."""
    tot = 0
    for t in TIER_NAMES:
        # tier statistics are global to the plan; take them from the first output's record
        tot += algorithmic_bytes(infos[0], t, s)
    return tot


def _same(C, D, rtol, what):
    a, b = C.to_host(), D.to_host()
    if not (np.array_equal(a.ptr, b.ptr) and np.array_equal(a.idx, b.idx)
            and (a.vid is None or np.array_equal(a.vid, b.vid))):
        raise AssertionError(f"{what}: patterns differ")
    if a.val is not None:
        if rtol == 0.0:
            ok = np.array_equal(a.val, b.val)
        else:
            ok = bool(np.all(np.abs(a.val - b.val) <= rtol * np.abs(b.val)))
        if not ok:
            raise AssertionError(f"{what}: values differ beyond {rtol}")


def _summa_diagnose(res, sg, dA, dB, sr):
    """On a mismatch: the differing columns, and which of the two forms a third one
    (the fused plan run as per-tier launches) agrees with on them."""
    from paper_1006_2183_amd import batched as BT
    third = BT.summa_share(sr, dA, dB, batched=False).to_host()
    C = {k: v.to_host() for k, v in res.items()}
    C["per_tier"] = third
    cols = {k: {int(H.vid[t]): H.idx[H.ptr[t]:H.ptr[t + 1]] for t in range(len(H.vid))} for k, H in C.items()}
    none = np.zeros(0, np.int32)
    allj = set(cols["plain"]) | set(cols["batched"]) | set(cols["per_tier"])
    bad = sorted(j for j in allj if not (np.array_equal(cols["plain"].get(j, none), cols["batched"].get(j, none))
                                         and np.array_equal(cols["plain"].get(j, none), cols["per_tier"].get(j, none))))
    odd = {k: sum(1 for j in bad if not np.array_equal(cols[k].get(j, none), cols["per_tier"].get(j, none)))
           for k in ("plain", "batched")}
    return f"{len(bad)} columns differ (first {bad[:5]}); columns where each form differs from the per-tier run: {odd}"


def suite_small(sg, torch, W, reps=50):
    """The small plain product (R-MAT scale 10, edge factor 8): latency-bound, so its
    time per product (symbolic + numeric) and per graph replay of the numeric launch."""
    from paper_1006_2183_amd import batched as BT
    out = {"workload": "rmat_s10_ef8_AxA_plain"}
    for sr in ("plus_times_f64", "min_plus_i32"):
        A = W.rmat_matrix(10, 8, sr, "csr", seed=1, abcd=RMAT_ABCD)
        dA = sg.DevMat.from_host(A, "cuda", sr)
        def step():
            sg.spgemm(sr, dA, dA)
        step()
        ms = _median_ms(torch, step, reps)
        plan = sg.spgemm_symbolic(sr, [dA], [dA])
        G = BT.GraphedNumeric(plan)
        G.replay()
        torch.cuda.synchronize()
        ms_graph = _median_ms(torch, G.replay, reps)
        info = plan.infos[0]
        plan.destroy()
        out[sr] = {"flops": info["flops"], "nnz_C": info["nnz"], "product_ms": round(ms, 4),
                   "graph_replay_ms": round(ms_graph, 4)}
        # the oracle on the same product, one thread (median of 5)
        import oracle
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            oracle.spgemm(sr, A, A)
            ts.append((time.perf_counter() - t0) * 1e3)
        out[sr]["cpu_baseline"] = {"value": round(sorted(ts)[2], 4), "unit": "ms per product", "cores": 1,
                                   "kind": "oracle", "sample": "the whole product, median of 5 runs"}
    return out


def suite_summa(sg, torch, W, reps, scale=24, grid=64, seed=24):
    """One Sparse SUMMA process's share: 64 stage products of DCSC blocks, merged."""
    from paper_1006_2183_amd import batched as BT
    sr = "plus_times_f64"
    log(f"[bench] SUMMA share: R-MAT scale {scale}, {grid}x{grid} grid, process (0,0)")
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (0, 0), semiring=sr, seed=seed, device="cuda", fmt="dcsc")
    dA = [sg.DevMat.from_host(x, "cuda", sr) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", sr) for x in b_blocks]
    nnz_blocks = [x.nnz for x in a_blocks]
    cpu = summa_cpu_baseline(sr, a_blocks, b_blocks, grid, (1 << scale) // grid)
    del a_blocks, b_blocks
    torch.cuda.empty_cache()
    res = {}

    def plain():
        parts = [sg.spgemm(sr, a, b, out_fmt="dcsc") for a, b in zip(dA, dB)]
        res["plain"] = BT.merge_partials(sr, parts)

    def batched():
        res["batched"] = BT.summa_share(sr, dA, dB, batched=True)

    plain()
    batched()
    try:
        _same(res["batched"], res["plain"], 1e-12, "SUMMA batched vs plain")
    except AssertionError as e:
        raise AssertionError(f"{e}; {_summa_diagnose(res, sg, dA, dB, sr)}")
    # the replayed plan's setting comes from the tuner, timing the persistent
    # launch alone (the replayed form): joint presets (entry records, mid-tier
    # capacity), then a coordinate descent over the record budget and the
    # tier thresholds
    from paper_1006_2183_amd import autotune as AT
    tune = AT.autotune(sr, dA, dB, [0] * len(dA), 1, out_fmt="dcsc", form="numeric_reuse", reps=3,
                       space=AT.REPLAY_SPACE, presets=AT.REPLAY_PRESETS)
    replay_tuning = tune["tuning"]
    log(f"[bench] SUMMA replay tuning {replay_tuning}: {tune['ms']:.3f} ms per launch "
        f"(default {tune['default_ms']:.3f} ms, {tune['tried']} settings)")
    plan = BT.summa_share_plan(sr, dA, dB, tuning=sg.make_tuning(sr, **replay_tuning))
    flops = sum(i["flops"] for i in plan.infos)
    nnz_c = plan.infos[0]["nnz"]
    G = BT.GraphedNumeric(plan)
    G.replay()
    torch.cuda.synchronize()
    # FP64 sums accumulate through LDS atomics, so two runs may round differently
    _same(G.outputs[0], res["batched"], 1e-12, "SUMMA graph replay vs batched")
    ms_plain = _median_ms(torch, plain, reps)
    ms_batched = _median_ms(torch, batched, reps)
    ms_graph = _median_ms(torch, G.replay, max(reps, 5))
    plan.profile(True)
    sg.spgemm_batched(plan, G.outputs)
    kms = plan.kernel_times()["heavy"]
    algo = _tier_bytes(plan.infos, 8)
    out = {
        "workload": SUMMA_WORKLOAD,
        "stages": len(dA), "nnz_blocks_min": int(min(nnz_blocks)), "nnz_blocks_max": int(max(nnz_blocks)),
        "flops": int(flops), "nnz_C": int(nnz_c),
        "plain_ms": round(ms_plain, 3), "batched_ms": round(ms_batched, 3), "graph_replay_ms": round(ms_graph, 3),
        "plain_GFLOPs": round(flops / ms_plain / 1e6, 2), "batched_GFLOPs": round(flops / ms_batched / 1e6, 2),
        "graph_GFLOPs": round(flops / ms_graph / 1e6, 2), "graph_plan_tuning": replay_tuning,
        "tuner": {"form": "numeric_reuse", "settings_tried": tune["tried"], "default_launch_ms": round(tune["default_ms"], 3),
                  "tuned_launch_ms": round(tune["ms"], 3)},
        "batched_vs_plain": round(ms_plain / ms_batched, 2), "graph_vs_plain": round(ms_plain / ms_graph, 2),
        "persistent_kernel": {"launch_ms": round(kms, 4), "algorithmic_bytes": int(algo),
                              "achieved_GBs": round(algo / kms / 1e6, 1) if kms > 0 else None,
                              "kernels": "k_small (small list) then k_batched (all other tiers), one replay",
                              # counters are taken on the replay-only run at SUMMA_PROFILE_TUNING
                              "traffic": load_traffic("replay", SUMMA_WORKLOAD, sr)
                              if replay_tuning == SUMMA_PROFILE_TUNING else None},
        "plain": "64 x (symbolic + sync + alloc + per-tier numeric) into DCSC partials, then a 64-way merge",
        "exact": "batched == plain == graph replay (patterns exact, values within 1e-12 relative)",
        "cpu_baseline": cpu,
    }
    plan.destroy()
    del G, res, dA, dB
    torch.cuda.empty_cache()
    return out


SUMMA_WORKLOAD = "rmat_s24_ef16_summa64x64_share_p00_f64"
SUMMA_PROFILE_TUNING = {"entry_mb": 1024}  # the replay-only run's setting (kernel traces, counters)


def suite_summa_replay(sg, torch, W, reps, tuning, scale=24, grid=64, seed=24):
    """Graph replays of the SUMMA share's plan alone (no plain path, no tuner), so that
    a kernel trace or a counter pass sees only the replayed launches: the small-list
    kernel and the persistent kernel, once per replay."""
    from paper_1006_2183_amd import batched as BT
    sr = "plus_times_f64"
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (0, 0), semiring=sr, seed=seed, device="cuda", fmt="dcsc")
    dA = [sg.DevMat.from_host(x, "cuda", sr) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", sr) for x in b_blocks]
    del a_blocks, b_blocks
    plan = BT.summa_share_plan(sr, dA, dB, tuning=sg.make_tuning(sr, **tuning))
    G = BT.GraphedNumeric(plan)
    ms = _median_ms(torch, G.replay, reps)
    plan.profile(True)
    sg.spgemm_batched(plan, G.outputs)
    kms = plan.kernel_times()["heavy"]
    algo = _tier_bytes(plan.infos, 8)
    out = {"workload": SUMMA_WORKLOAD, "tuning": tuning, "replays": reps, "graph_replay_ms": round(ms, 3),
           "launch_ms": round(kms, 4), "algorithmic_bytes": int(algo),
           "n_small": plan.infos[0]["n_small"], "n_mid": plan.infos[0]["n_mid"]}
    plan.destroy()
    return out


GALERKIN_WORKLOAD = "galerkin_rap_7pt_16_instances_n_in_32_48_64_96_128_f64"


def galerkin_operands(sg, W, count=16, seed=4):
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.choice([32, 48, 64, 96, 128], size=count)]
    host = {}
    for n in sorted(set(sizes)):
        L = W.laplacian_7pt(n, "csr")
        P = W.aggregation_p(n, "csr")
        host[n] = (L, P, W.transpose(P, "csr"))
    dev = lambda M: sg.DevMat.from_host(M, "cuda")
    return sizes, host, [dev(host[n][0]) for n in sizes], [dev(host[n][1]) for n in sizes], \
        [dev(host[n][2]) for n in sizes]


def suite_galerkin_replay(sg, torch, W, reps):
    """Graph replays alone of the Galerkin batch's two-launch chain (A P, then R (A P),
    default settings) and of the fused chain, so that a counter pass sees only their
    numeric launches: `reps` replays of each after the one eager launch each graph's
    set-up runs."""
    from paper_1006_2183_amd import batched as BT
    sr = "plus_times_f64"
    sizes, host, Ls, Ps, Rs = galerkin_operands(sg, W)
    plan_ap, AP, plan_rap = BT.galerkin_plans(sr, Rs, Ls, Ps)
    G = BT.GraphedNumeric([plan_ap, plan_rap], [AP, None])
    for _ in range(reps):
        G.replay()
    torch.cuda.synchronize()
    plan_f = BT.galerkin_chain_plan(sr, Rs, Ls, Ps)
    GF = BT.GraphedNumeric(plan_f)
    for _ in range(reps):
        GF.replay()
    torch.cuda.synchronize()
    out = {"workload": GALERKIN_WORKLOAD, "replays": reps, "launches_each": reps + 1}
    plan_f.destroy()
    return out


def summa_cpu_baseline(sr, a_blocks, b_blocks, grid, b):
    """The oracle on the whole share: the strip product A(I, :) A(:, J)."""
    import oracle
    ra, ca, va, rb, cb, vb = [], [], [], [], [], []
    for k in range(grid):
        A, B = a_blocks[k], b_blocks[k]
        ra.append(A.idx.astype(np.int64)); va.append(A.val)
        ca.append(np.repeat(A.vid.astype(np.int64), np.diff(A.ptr)) + k * b)
        rb.append(B.idx.astype(np.int64) + k * b); vb.append(B.val)
        cb.append(np.repeat(B.vid.astype(np.int64), np.diff(B.ptr)))
    import workloads as W
    SA = W.from_triples(np.concatenate(ra), np.concatenate(ca), np.concatenate(va), b, grid * b, "dcsc", sr)
    SB = W.from_triples(np.concatenate(rb), np.concatenate(cb), np.concatenate(vb), grid * b, b, "dcsc", sr)
    fn = lambda th: oracle.spgemm(sr, SA, SB) if th == 1 else oracle.spgemm_threads(sr, SA, SB, threads=th)
    return cpu_rate(fn, "the whole share as one product of the DCSC strips A(I,:) A(:,J) (the block identity)")


def suite_galerkin(sg, torch, W, reps, count=16, seed=4):
    """R (A P) for uneven 3D Poisson instances, plain vs grouped vs graph, autotuned."""
    from paper_1006_2183_amd import batched as BT
    from paper_1006_2183_amd import autotune as AT
    sr = "plus_times_f64"
    sizes, host, Ls, Ps, Rs = galerkin_operands(sg, W, count, seed)
    log(f"[bench] Galerkin R A P: {count} instances, grid sizes {sizes}")
    res = {}

    def plain():
        res["plain"] = [sg.spgemm(sr, R, sg.spgemm(sr, L, P)) for R, L, P in zip(Rs, Ls, Ps)]

    def batched(tuning=None):
        res["batched"] = BT.galerkin_rap(sr, Rs, Ls, Ps, batched=True, tuning=tuning)

    plain()
    batched()
    for i, n in enumerate(sizes):
        _same(res["batched"][i], res["plain"][i], 0.0, f"Galerkin instance {i}")
        if i < len(set(sizes)) or i == count - 1:
            Lc = W.laplacian_7pt(n // 2, "csr")
            got = res["batched"][i].to_host()
            if not (np.array_equal(got.ptr, Lc.ptr) and np.array_equal(got.idx, Lc.idx)
                    and np.array_equal(got.val, 4.0 * Lc.val)):
                raise AssertionError(f"Galerkin instance {i}: R A P != 4 L_(n/2)")
    plan_ap, AP, plan_rap = BT.galerkin_plans(sr, Rs, Ls, Ps)
    flops = sum(i["flops"] for i in plan_ap.infos) + sum(i["flops"] for i in plan_rap.infos)
    # tune the two grouped products (the persistent launch), then time with the tuned setting
    t_ap = AT.autotune(sr, Ls, Ps, list(range(count)), count, form="batched", reps=2)
    t_rap = AT.autotune(sr, Rs, AP, list(range(count)), count, form="batched", reps=2)
    tun_ap = sg.make_tuning(sr, **t_ap["tuning"])
    tun_rap = sg.make_tuning(sr, **t_rap["tuning"])

    def tuned():
        APt = sg.spgemm_grouped(sr, Ls, Ps, list(range(count)), count, tuning=tun_ap, batched=True)
        res["tuned"] = sg.spgemm_grouped(sr, Rs, APt, list(range(count)), count, tuning=tun_rap, batched=True)

    tuned()
    for i in range(count):
        _same(res["tuned"][i], res["plain"][i], 0.0, f"Galerkin tuned instance {i}")
    G = BT.GraphedNumeric([plan_ap, plan_rap], [AP, None])
    G.replay()
    torch.cuda.synchronize()
    for i in range(count):
        _same(G.outputs[i], res["plain"][i], 0.0, f"Galerkin graph instance {i}")
    # fused chain: one plan, A P never written; its symbolic phase is reused by replays
    plan_f = BT.galerkin_chain_plan(sr, Rs, Ls, Ps)
    GF = BT.GraphedNumeric(plan_f)
    GF.replay()
    torch.cuda.synchronize()
    for i in range(count):
        _same(GF.outputs[i], res["plain"][i], 0.0, f"Galerkin fused graph instance {i}")

    def fused():
        res["fused"] = BT.galerkin_fused(sr, Rs, Ls, Ps, batched=True)

    fused()
    for i in range(count):
        _same(res["fused"][i], res["plain"][i], 0.0, f"Galerkin fused instance {i}")
    ms_plain = _median_ms(torch, plain, reps)
    ms_batched = _median_ms(torch, batched, reps)
    ms_tuned = _median_ms(torch, tuned, reps)
    ms_graph = _median_ms(torch, G.replay, max(reps, 5))
    ms_fused = _median_ms(torch, fused, reps)
    ms_fgraph = _median_ms(torch, GF.replay, max(reps, 5))
    plan_f.profile(True)
    sg.spgemm_batched(plan_f, GF.outputs)
    kt = plan_f.kernel_times()
    flops_f = sum(i["flops"] for i in plan_f.infos)
    nnz_f = sum(i["nnz"] for i in plan_f.infos)
    # algorithmic bytes of the fused launch: stream P (4 + 8 per entry, 8 per
    # pointer), the pointer pair of every gathered A and R vector, gather the
    # entries of both stages (12 per multiplication), write R A P (12 per entry)
    nnzP = sum(int(P.nnz) for P in Ps)
    nvecP = sum(int(P.nvec) for P in Ps)
    algo_f = 12 * nnzP + 8 * nvecP + 16 * flops_f // 4 + 12 * flops_f + 12 * nnz_f
    launch_f = kt["tiny"] + kt["mid"]
    out_fused = {"graph_replay_ms": round(ms_fgraph, 3), "plan_and_numeric_ms": round(ms_fused, 3),
                 "flops": int(flops_f), "graph_GFLOPs": round(flops_f / ms_fgraph / 1e6, 2),
                 "graph_vs_two_launch_graph": round(ms_graph / ms_fgraph, 2),
                 "tiers": {"tiny": plan_f.infos[0]["n_tiny"], "mid": plan_f.infos[0]["n_mid"]},
                 "launch_ms": round(launch_f, 4),
                 "algorithmic_bytes": int(algo_f),
                 "achieved_GBs": round(algo_f / launch_f / 1e6, 1) if launch_f > 0 else None,
                 "traffic": load_traffic("fused_replay", GALERKIN_WORKLOAD, sr),
                 "exact": "fused == plain bitwise (R A P == 4 L_(n/2) on every instance)"}
    plan_f.destroy()
    out = {
        "workload": GALERKIN_WORKLOAD,
        "graph_replay_traffic": load_traffic("two_launch_replay", GALERKIN_WORKLOAD, sr),
        "fused_chain": out_fused,
        "sizes": sizes, "flops": int(flops),
        "nnz_RAP": int(sum(i["nnz"] for i in plan_rap.infos)),
        "plain_ms": round(ms_plain, 3), "batched_ms": round(ms_batched, 3), "tuned_ms": round(ms_tuned, 3),
        "graph_replay_ms": round(ms_graph, 3),
        "plain_GFLOPs": round(flops / ms_plain / 1e6, 2), "batched_GFLOPs": round(flops / ms_batched / 1e6, 2),
        "tuned_GFLOPs": round(flops / ms_tuned / 1e6, 2), "graph_GFLOPs": round(flops / ms_graph / 1e6, 2),
        "batched_vs_plain": round(ms_plain / ms_batched, 2), "graph_vs_plain": round(ms_plain / ms_graph, 2),
        "autotune": {"ap": {"tuning": t_ap["tuning"], "ms": round(t_ap["ms"], 3),
                            "default_ms": round(t_ap["default_ms"], 3), "tried": t_ap["tried"]},
                     "rap": {"tuning": t_rap["tuning"], "ms": round(t_rap["ms"], 3),
                             "default_ms": round(t_rap["default_ms"], 3), "tried": t_rap["tried"]}},
        "plain": "per instance: symbolic + sync + alloc + numeric for A P, then for R (A P)",
        "exact": "plain == grouped == tuned == graph bitwise; R A P == 4 L_(n/2) checked on one instance per size",
    }
    import oracle

    def cpu_fn(th):
        fl = 0
        for n in sizes:
            L, P, R = host[n]
            mul = (lambda a, b: oracle.spgemm(sr, a, b)) if th == 1 else \
                (lambda a, b: oracle.spgemm_threads(sr, a, b, threads=th))
            AP_, f1 = mul(L, P)
            _, f2 = mul(R, AP_)
            fl += f1 + f2
        return None, fl

    out["cpu_baseline"] = cpu_rate(cpu_fn, f"all {count} instances, each as two oracle calls A P then R (A P)")
    plan_ap.destroy()
    plan_rap.destroy()
    del G, res, Ls, Ps, Rs, AP
    torch.cuda.empty_cache()
    return out


def suite_serve(sg, torch, W, count, qps_list, scale=20, seed=1):
    """Served multi-source expansions Y = A X ((or, and)), Poisson arrivals; batched server vs FIFO.

    Requests arrive as host frontiers (one source per column); both servers build
    the sparse operand on the device. The batched server concatenates a batch's
    frontiers into one operand and runs one product per batch on two streams;
    FIFO runs one plain product per request."""
    from paper_1006_2183_amd import serve as SV
    sr = "or_and_bool"
    log(f"[bench] serving: R-MAT scale {scale} bool resident, {count} requests per QPS level {qps_list}")
    A = W.rmat_matrix(scale, 16, sr, "csc", seed=seed, device="cuda")
    dA = sg.DevMat.from_host(A, "cuda", sr)
    colcount = np.diff(A.ptr)
    rng = np.random.default_rng(seed + 100)
    ks = rng.integers(1, 513, size=count)
    fronts, srcs = [], []
    for i, k in enumerate(ks):
        src = np.random.default_rng(1000 + i).integers(0, A.nrows, size=int(k))
        fronts.append(SV.Frontier.sources(src))
        srcs.append(src.astype(np.int64))  # depth 0: X(:, s) holds only source s
    ubs = [SV.frontier_bound(colcount, f) for f in fronts]
    out = {"workload": f"rmat_s{scale}_ef16_bool_csc_resident_bfs_depth0_k_U1_512", "requests": count,
           "request_flops_p50": float(np.percentile(ubs, 50)), "request_flops_p99": float(np.percentile(ubs, 99)),
           "operand_build": "on the device from the request's host triples (sg_coo_compress / sg_coo_emit)",
           "levels": []}
    # warm both paths
    for ex in (SV.FrontierBatchExecutor(dA), SV.FrontierFifoExecutor(dA)):
        SV.Scheduler(ex, 1 << 26).run([SV.Request(0, 0.0, fronts[0], ubs[0])])
    torch.cuda.synchronize()

    def check(done):
        # depth-0 closed form: Y(:, s) is the pattern of A(:, src_s)
        for r in done:
            Y = (r.result[0] if isinstance(r.result, list) else r.result).to_host()
            src = srcs[r.rid]
            for s_ in range(len(src)):
                ref = A.idx[A.ptr[src[s_]]:A.ptr[src[s_] + 1]]
                if not np.array_equal(Y.idx[Y.ptr[s_]:Y.ptr[s_ + 1]], ref):
                    raise AssertionError(f"request {r.rid} column {s_} differs from A(:, src)")

    for qps in qps_list:
        arr = W.poisson_arrivals(qps, count, seed=int(qps))
        line = {"qps": qps}
        for name, ex, mb in (("batched", SV.FrontierBatchExecutor(dA), 64), ("fifo", SV.FrontierFifoExecutor(dA), 1)):
            reqs = [SV.Request(i, float(arr[i]), fronts[i], ubs[i]) for i in range(count)]
            sched = SV.Scheduler(ex, pool_entries=1 << 26, max_batch=mb, max_inflight=2 if mb > 1 else 1)
            done = sched.run(reqs)
            torch.cuda.synchronize()
            if len(done) != count:
                raise AssertionError(f"{name} server finished {len(done)} of {count} requests")
            st = SV.latency_stats(done)
            check([r for r in done if r.status == "done"])
            line[name] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
            line[name]["launches"] = sched.batches
            log(f"[bench] serving qps {qps} {name}: {line[name]}")
        out["levels"].append(line)
    out["exact"] = "every served column equals the pattern of A(:, src) (depth-0 closed form), both servers"
    import oracle
    import concurrent.futures as cf
    hostX = [W.from_triples(f.rows, f.cols, None, A.nrows, f.k, "csc", sr) for f in fronts]

    def cpu_fn(th):
        if th == 1:
            return None, sum(oracle.spgemm(sr, A, X)[1] for X in hostX)
        with cf.ThreadPoolExecutor(max_workers=th) as ex:
            return None, sum(f for _, f in ex.map(lambda X: oracle.spgemm(sr, A, X), hostX))

    cb = cpu_rate(cpu_fn, f"all {count} requests Y = A X, one oracle call each (requests spread over the threads)")
    cb["requests_per_s"] = round(count / cb["seconds"]["all_cores"], 1)
    cb["requests_per_s_single_thread"] = round(count / cb["seconds"]["single_thread"], 1)
    out["cpu_baseline"] = cb
    del dA
    torch.cuda.empty_cache()
    return out


def suite_bfs(sg, torch, W, count, qps_list, scale=20, seed=1, kmax=32, max_levels=3):
    """Served masked multi-level BFS (Section 6.2.2): requests of k ~ U[1, kmax] random
    sources, each searched to depth max_levels (frontier loop: one masked product per
    level, visited bitmaps updated on the device). Iteration-level batching (every
    iteration one grouped masked product over all active requests, at mixed depths)
    against a FIFO server (one request at a time, one plain masked product per level)."""
    from paper_1006_2183_amd import bfs as BF
    import oracle.bfs as OB
    sr = "or_and_bool"
    log(f"[bench] BFS serving: R-MAT scale {scale} bool, {count} requests per QPS level {qps_list}")
    A = W.rmat_matrix(scale, 16, sr, "csc", seed=seed, device="cuda")
    dA = sg.DevMat.from_host(A, "cuda", sr)
    rng = np.random.default_rng(seed + 200)
    ks = rng.integers(1, kmax + 1, size=count)
    srcs = [np.random.default_rng(3000 + i).integers(0, A.nrows, size=int(k)) for i, k in enumerate(ks)]
    out = {"workload": f"rmat_s{scale}_ef16_bool_csc_masked_bfs_k_U1_{kmax}_depth{max_levels}", "requests": count,
           "levels": []}
    # warm-up
    BF.BfsServer(dA).run([BF.BfsRequest(0, 0.0, srcs[0], max_levels)])
    torch.cuda.synchronize()
    checked = 0
    for qps in qps_list:
        arr = W.poisson_arrivals(qps, count, seed=int(qps) + 1)
        line = {"qps": qps}
        for name, batched in (("batched", True), ("fifo", False)):
            reqs = [BF.BfsRequest(i, float(arr[i]), srcs[i], max_levels) for i in range(count)]
            srv = BF.BfsServer(dA, pool_bytes=16 << 30, max_active=64, batched=batched)
            done = srv.run(reqs)
            torch.cuda.synchronize()
            st = BF.bfs_latency(done)
            line[name] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
            line[name]["iterations"] = srv.iterations
            if batched:
                mixes = [len(m) for m in srv.mix]
                line[name]["active_per_iteration_mean"] = round(float(np.mean([sum(m.values()) for m in srv.mix])), 2)
                line[name]["iterations_with_mixed_depths"] = int(sum(1 for x in mixes if x > 1))
            # the first few requests of the run, level by level, against the oracle's BFS
            for r in sorted(done, key=lambda r: r.rid)[:3]:
                want = OB.bfs_levels(A, r.sources, max_levels=max_levels)
                got = [Y.to_host() for Y in r.levels]
                if len(got) != max(len(w) for w in want):
                    raise AssertionError(f"BFS request {r.rid}: depth differs")
                for d, Y in enumerate(got):
                    for c in range(len(r.sources)):
                        exp = want[c][d] if d < len(want[c]) else np.zeros(0, np.int64)
                        if not np.array_equal(Y.idx[Y.ptr[c]:Y.ptr[c + 1]], exp):
                            raise AssertionError(f"BFS request {r.rid} level {d} column {c} differs from the oracle")
                checked += 1
            log(f"[bench] BFS qps {qps} {name}: {line[name]}")
            del done, reqs
        out["levels"].append(line)
    out["exact"] = f"{checked} served requests checked level by level against the oracle's BFS (bit-exact)"
    # CPU baseline: the oracle's BFS (plain Python, one thread) on the first
    # requests, as many as fit about 10 s
    t0 = time.perf_counter()
    nreq = nsrc = 0
    while nreq < count and (nreq == 0 or time.perf_counter() - t0 < 10.0):
        OB.bfs_levels(A, srcs[nreq], max_levels=max_levels)
        nsrc += len(srcs[nreq])
        nreq += 1
    dt = time.perf_counter() - t0
    out["cpu_baseline"] = {"value": round(nreq / dt, 4), "unit": "requests/s", "cores": 1, "kind": "oracle",
                           "sources_per_s": round(nsrc / dt, 3), "host": host_info(),
                           "sample": f"the first {nreq} requests ({nsrc} sources, depth {max_levels}), one "
                                     f"level-set search per source in plain Python, {dt:.1f} s"}
    del dA
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# Counter ingestion: HBM bytes per launch from rocprofv3 --pmc passes

def _counter_rows(d):
    """(kernel name, counter name, value) of every dispatch in a rocprofv3 --pmc CSV under d."""
    import csv
    rows = []
    for dirpath, _, files in os.walk(d):
        for f in files:
            if f.endswith("counter_collection.csv"):
                with open(os.path.join(dirpath, f)) as fh:
                    for r in csv.DictReader(fh):
                        rows.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]),
                                     r.get("Dispatch_Id", "")))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def ingest_counters(root, copy_mib, workload, semiring):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the numeric heavy kernel by the
    ratio the same counters read for a device copy of known size; write profiles/hbm_traffic.json."""
    import re
    copy_bytes = copy_mib * (1 << 20)
    factors = {}
    for ctr, sub in (("FETCH_SIZE", "cal_fetch"), ("WRITE_SIZE", "cal_write")):
        vals = [v for k, c, v, _ in _counter_rows(os.path.join(root, sub)) if c == ctr and "copy" in k.lower()]
        if not vals:
            raise SystemExit(f"no copy kernel dispatch in {sub}")
        factors[ctr] = copy_bytes / (float(np.median(vals)) * 1024.0)
    per = {}
    pat = re.compile(r"k_heavy<\d+, \d+(, (true|false))?>")  # the numeric heavy kernel (not k_heavy_count)
    for ctr, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        vals = [v for k, c, v, _ in _counter_rows(os.path.join(root, sub)) if c == ctr and pat.search(k)]
        if not vals:
            raise SystemExit(f"no numeric k_heavy dispatch in {sub}")
        per[ctr] = float(np.mean(vals)) * 1024.0 * factors[ctr]
    entry = {"kernel_hash": kernel_source_hash(), "bytes_per_launch": int(per["FETCH_SIZE"] + per["WRITE_SIZE"]),
             "fetch_bytes": int(per["FETCH_SIZE"]), "write_bytes": int(per["WRITE_SIZE"]),
             "copy_scale": {k: round(v, 4) for k, v in factors.items()}, "copy_mib": copy_mib}
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    d = {}
    if os.path.exists(path):
        with open(path) as f:
            d = json.load(f)
    d[f"{workload}/{semiring}/k_heavy"] = entry
    # the SUMMA share's replayed launch (k_small and the persistent kernel, counted
    # together per replay) when its passes were taken too
    if os.path.isdir(os.path.join(root, "summa_fetch")):
        sp = {}
        pats = (re.compile(r"k_batched<\d+, \d+, true>"), re.compile(r"k_small<\d+, false, true>"))
        for ctr, sub in (("FETCH_SIZE", "summa_fetch"), ("WRITE_SIZE", "summa_write")):
            rows = [(k, v) for k, c, v, _ in _counter_rows(os.path.join(root, sub)) if c == ctr]
            tot = 0.0
            for pt in pats:
                vals = [v for k, v in rows if pt.search(k)]
                tot += float(np.mean(vals)) if vals else 0.0
            if not any(pats[0].search(k) for k, _ in rows):
                raise SystemExit(f"no persistent-kernel dispatch in {sub}")
            sp[ctr] = tot * 1024.0 * factors[ctr]
        se = {"kernel_hash": kernel_source_hash(), "bytes_per_launch": int(sp["FETCH_SIZE"] + sp["WRITE_SIZE"]),
              "fetch_bytes": int(sp["FETCH_SIZE"]), "write_bytes": int(sp["WRITE_SIZE"]),
              "copy_scale": {k: round(v, 4) for k, v in factors.items()}, "copy_mib": copy_mib}
        d[f"{SUMMA_WORKLOAD}/plus_times_f64/replay"] = se
        print(json.dumps(se))
    # the Galerkin batch's replays: the fused chain (k_chain_tiny / k_chain_mid per
    # launch) and the two-launch chain (two k_tiny launches per replay)
    if os.path.isdir(os.path.join(root, "galerkin_fetch")):
        def two_sizes(vals):
            # the two launches of a replay (A P, then R (A P)) differ in size: the
            # median of each of the two clusters of dispatch values, added
            lo, hi = min(vals), max(vals)
            cut = (lo + hi) / 2.0
            big = [v for v in vals if v > cut] or [hi]
            small = [v for v in vals if v <= cut] or [lo]
            return float(np.median(big)) + float(np.median(small))

        for key, pats, two in (("fused_replay", (re.compile(r"k_chain_tiny<\d+, false>"),
                                                 re.compile(r"k_chain_mid<\d+, false>")), False),
                               ("two_launch_replay", (re.compile(r"k_tiny<\d+, false>"),), True)):
            gp = {}
            for ctr, sub in (("FETCH_SIZE", "galerkin_fetch"), ("WRITE_SIZE", "galerkin_write")):
                rows = [(k, v) for k, c, v, _ in _counter_rows(os.path.join(root, sub)) if c == ctr]
                tot = 0.0
                for pt in pats:
                    vals = [v for k, v in rows if pt.search(k)]
                    if vals:
                        tot += two_sizes(vals) if two else float(np.median(vals))
                gp[ctr] = tot * 1024.0 * factors[ctr]
            ge = {"kernel_hash": kernel_source_hash(), "bytes_per_launch": int(gp["FETCH_SIZE"] + gp["WRITE_SIZE"]),
                  "fetch_bytes": int(gp["FETCH_SIZE"]), "write_bytes": int(gp["WRITE_SIZE"]),
                  "copy_scale": {k: round(v, 4) for k, v in factors.items()}, "copy_mib": copy_mib}
            d[f"{GALERKIN_WORKLOAD}/plus_times_f64/{key}"] = ge
            print(key, json.dumps(ge))
    with open(path, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print(json.dumps(entry))


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
    ap.add_argument("--no-suite", action="store_true",
                    help="skip the batched (SUMMA share, Galerkin) and served measurements")
    ap.add_argument("--suite-reps", type=int, default=3)
    ap.add_argument("--only", choices=["small", "summa", "galerkin", "serving", "bfs", "summa_replay", "galerkin_replay"],
                    default=None,
                    help="run one of the batched/served measurements alone and print its JSON object")
    ap.add_argument("--serve-requests", type=int, default=600)
    ap.add_argument("--serve-qps", default="500,2000,8000")
    ap.add_argument("--bfs-requests", type=int, default=120)
    ap.add_argument("--bfs-qps", default="50,200")
    ap.add_argument("--ingest-counters", default=None,
                    help="directory holding fetch/, write/, cal_fetch/, cal_write/ rocprofv3 --pmc outputs: "
                         "write the measured HBM bytes per heavy launch to profiles/hbm_traffic.json and exit")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="run only a device copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()

    if args.ingest_counters:
        ingest_counters(args.ingest_counters, args.copy_mib, f"rmat_s{args.scale}_ef{args.edge_factor}_AxA_plain",
                        args.semiring)
        return

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

    suites = {"small": ("small_product", lambda: suite_small(sg, torch, W)),
              "summa": ("batched_summa", lambda: suite_summa(sg, torch, W, args.suite_reps)),
              "galerkin": ("batched_galerkin", lambda: suite_galerkin(sg, torch, W, args.suite_reps)),
              "serving": ("serving", lambda: suite_serve(sg, torch, W, args.serve_requests,
                                                         [float(q) for q in args.serve_qps.split(",")])),
              "bfs": ("served_bfs", lambda: suite_bfs(sg, torch, W, args.bfs_requests,
                                                      [float(q) for q in args.bfs_qps.split(",")])),
              "galerkin_replay": ("galerkin_replay", lambda: suite_galerkin_replay(sg, torch, W, args.suite_reps)),
              "summa_replay": ("summa_replay", lambda: suite_summa_replay(
                  sg, torch, W, args.suite_reps, json.loads(args.tuning) if args.tuning else SUMMA_PROFILE_TUNING))}
    if args.only:
        print(json.dumps({suites[args.only][0]: suites[args.only][1]()}), flush=True)
        return

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
    if not args.no_suite:
        for key, (name, fn) in suites.items():
            if key.endswith("_replay"):  # profiling runs of their own (--only), not part of the line
                continue
            t = time.perf_counter()
            try:
                out[name] = fn()
            except (AssertionError, sg.SgError, RuntimeError) as e:
                out[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] {name}: {time.perf_counter() - t:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
