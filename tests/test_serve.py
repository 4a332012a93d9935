"""Serving loop: host-side scheduling on the CPU with a fake executor and clock,
and (GPU) each request's result is the same alone and in the mix."""
import numpy as np
import pytest

import workloads as W
from paper_1006_2183_amd.serve import Request, Scheduler, frontier_bound, latency_stats


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """A batch takes `base + per_entry * sum(ub)` seconds of fake time."""

    def __init__(self, clock, base=1e-4, per_entry=1e-8):
        self.clock = clock
        self.base = base
        self.per_entry = per_entry
        self.inflight = []
        self.max_inflight_entries = 0
        self.max_overlap = 0
        self.launches = []

    def launch(self, batch):
        start = self.clock()
        end = start + self.base + self.per_entry * sum(r.ub for r in batch)
        h = (end, [r.rid for r in batch], sum(r.ub for r in batch))
        self.inflight.append(h)
        self.launches.append((start, end, tuple(r.rid for r in batch)))
        self.max_inflight_entries = max(self.max_inflight_entries, sum(x[2] for x in self.inflight))
        self.max_overlap = max(self.max_overlap, len(self.inflight))
        return h

    def poll(self, h):
        return self.clock() >= h[0]

    def finish(self, h):
        self.inflight.remove(h)
        return [("result", rid) for rid in h[1]]


def make_requests(n, qps, seed, ub_lo=100, ub_hi=5000, deadline=None):
    arr = W.poisson_arrivals(qps, n, seed)
    rng = np.random.default_rng(seed + 1)
    ubs = rng.integers(ub_lo, ub_hi, size=n)
    return [Request(i, float(arr[i]), None, int(ubs[i]), None if deadline is None else float(arr[i] + deadline))
            for i in range(n)]


def run_fake(reqs, pool, max_batch=16, max_inflight=2, step=5e-6):
    clock = FakeClock()
    ex = FakeExecutor(clock)

    def idle():
        clock.t += step

    sched = Scheduler(ex, pool, max_batch=max_batch, max_inflight=max_inflight, clock=clock, idle=idle)
    done = sched.run(reqs)
    return done, ex, sched


def test_all_requests_complete_with_nonnegative_latency():
    reqs = make_requests(300, 20000, 3)
    done, ex, sched = run_fake(reqs, pool=200000)
    assert len(done) == 300 and all(r.status == "done" for r in done)
    assert all(r.done >= r.arrival for r in done)
    assert all(r.result == ("result", r.rid) for r in done)
    st = latency_stats(done)
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_admission_never_exceeds_pool():
    reqs = make_requests(400, 50000, 5)
    pool = 12000
    done, ex, sched = run_fake(reqs, pool=pool)
    assert ex.max_inflight_entries <= pool
    assert sched.free == pool  # everything returned


def test_oversized_request_rejected_and_deadline_cancels():
    reqs = make_requests(50, 10000, 7)
    reqs[10].ub = 10 ** 9
    done, ex, sched = run_fake(reqs, pool=100000)
    st = {r.rid: r.status for r in done}
    assert st[10] == "rejected"
    assert sum(s == "done" for s in st.values()) == 49
    # a burst with a tight deadline and a slow executor: late requests are cancelled before launch
    reqs = make_requests(200, 10 ** 7, 9, ub_lo=40000, ub_hi=50000, deadline=2e-4)
    done, ex, sched = run_fake(reqs, pool=100000, max_batch=2, max_inflight=1)
    st = latency_stats(done)
    assert st["cancelled"] > 0 and st["done"] > 0 and st["done"] + st["cancelled"] == 200
    launched = {rid for _, _, b in ex.launches for rid in b}
    assert all(r.rid not in launched for r in done if r.status == "cancelled")


def test_continuous_batching_overlaps_batches():
    # arrivals keep coming while batches run: the next batch launches before the previous completes
    reqs = make_requests(500, 200000, 11)
    done, ex, sched = run_fake(reqs, pool=10 ** 7, max_batch=8, max_inflight=2)
    assert ex.max_overlap == 2
    overlapping = sum(1 for (s0, e0, _), (s1, e1, _) in zip(ex.launches, ex.launches[1:]) if s1 < e0)
    assert overlapping > 0
    # arrival order is kept within and across batches
    order = [rid for _, _, b in ex.launches for rid in b]
    assert order == sorted(order)


class CallbackExecutor(FakeExecutor):
    """Calls the scheduler back in the middle of every launch, as the GPU executors
    do between their host-blocking steps."""

    def __init__(self, clock):
        super().__init__(clock)
        self.between = None

    def launch(self, batch):
        self.clock.t += 3e-5  # planning time, during which earlier batches may end
        if self.between is not None:
            self.between()
        return super().launch(batch)


def test_callbacks_during_launch_lose_no_request():
    """Batches retired from inside a launch's callback leave the new batch in flight:
    every request completes exactly once."""
    clock = FakeClock()
    ex = CallbackExecutor(clock)

    def idle():
        clock.t += 5e-6

    reqs = make_requests(400, 20000.0, seed=8)
    done = Scheduler(ex, 1 << 30, max_batch=4, max_inflight=2, clock=clock, idle=idle).run(reqs)
    assert len(done) == len(reqs) and all(r.status == "done" for r in done)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert not ex.inflight


def test_deterministic_replay():
    a, ex_a, _ = run_fake(make_requests(200, 30000, 13), pool=50000)
    b, ex_b, _ = run_fake(make_requests(200, 30000, 13), pool=50000)
    assert ex_a.launches == ex_b.launches
    assert [(r.rid, r.done) for r in a] == [(r.rid, r.done) for r in b]


def test_frontier_bound_is_flops():
    A = W.rmat_matrix(9, 8, "or_and_bool", "csc", seed=2)
    X = W.bfs_frontier(A.nrows, 20, seed=3)
    colcount = np.diff(A.ptr)
    import oracle
    _, flops = oracle.spgemm("or_and_bool", A, X)
    assert frontier_bound(colcount, X) == flops


@pytest.mark.gpu
def test_gpu_alone_equals_mix():
    """Each request's result is bit-identical alone (one plain product) and inside
    continuously batched launches, and equals the oracle."""
    import torch
    import oracle
    import paper_1006_2183_amd as sg
    from paper_1006_2183_amd.serve import GpuBatchExecutor
    from tests.helpers import assert_same
    sg.load_library()
    A = W.rmat_matrix(12, 16, "or_and_bool", "csc", seed=1)
    dA = sg.DevMat.from_host(A, "cuda", "or_and_bool")
    colcount = np.diff(A.ptr)
    rng = np.random.default_rng(4)
    hostX = []
    reqs = []
    arr = W.poisson_arrivals(4000.0, 60, 6)
    for i in range(60):
        k = int(rng.integers(1, 65))
        X = W.bfs_frontier(A.nrows, k, seed=100 + i, A=A, depth=int(i % 3 == 0))
        hostX.append(X)
        reqs.append(Request(i, float(arr[i]), sg.DevMat.from_host(X, "cuda", "or_and_bool"), frontier_bound(colcount, X)))
    ex = GpuBatchExecutor("or_and_bool", dA)
    sched = Scheduler(ex, pool_entries=1 << 24, max_batch=8, max_inflight=2)
    done = sched.run(reqs)
    torch.cuda.synchronize()
    assert all(r.status == "done" for r in done)
    assert sched.batches < 60  # requests were batched
    for r in sorted(done, key=lambda r: r.rid):
        mix = r.result.to_host()
        alone = sg.spgemm("or_and_bool", dA, r.X).to_host()
        assert np.array_equal(mix.ptr, alone.ptr) and np.array_equal(mix.idx, alone.idx), f"request {r.rid}"
        if r.rid % 10 == 0:
            R, _ = oracle.spgemm("or_and_bool", A, hostX[r.rid])
            assert_same(mix, R, "or_and_bool")
    print(latency_stats(done), flush=True)



@pytest.mark.gpu
def test_gpu_two_batches_in_flight():
    """Continuous batching overlaps batches on the device: a second batch is planned
    and launched on the other stream while the first one's launch is still running
    (its start event precedes the first batch's end event), and both results equal
    the requests computed alone."""
    import torch
    import paper_1006_2183_amd as sg
    from paper_1006_2183_amd.serve import GpuBatchExecutor
    sg.load_library()
    # the first batch holds about 270 M multiplications (several ms on the device), so
    # the host plans and launches the second one while it runs
    A = W.rmat_matrix(18, 16, "or_and_bool", "csc", seed=2)
    dA = sg.DevMat.from_host(A, "cuda", "or_and_bool")
    colcount = np.diff(A.ptr)
    heavy = [W.bfs_frontier(A.nrows, 512, seed=300 + i, A=A, depth=1) for i in range(48)]
    light = [W.bfs_frontier(A.nrows, 4, seed=400 + i) for i in range(4)]
    mk = lambda i, X: Request(i, 0.0, sg.DevMat.from_host(X, "cuda", "or_and_bool"), frontier_bound(colcount, X))
    b1 = [mk(i, X) for i, X in enumerate(heavy)]
    b2 = [mk(100 + i, X) for i, X in enumerate(light)]
    ex = GpuBatchExecutor("or_and_bool", dA, timing=True)
    # warm-up (kernel loading, allocator)
    ex.finish(ex.launch(b2))
    torch.cuda.synchronize()
    ex.intervals.clear()
    h1 = ex.launch(b1)
    h2 = ex.launch(b2)
    torch.cuda.synchronize()
    (s1, a1, e1), (s2, a2, e2) = ex.intervals
    assert s1 != s2
    gap = e1.elapsed_time(a2)  # negative: batch 2 started before batch 1 ended
    print(f"batch 1 {a1.elapsed_time(e1):.3f} ms, batch 2 starts {gap:.3f} ms after batch 1 ends", flush=True)
    assert gap < 0, "the second batch did not start while the first was in flight"
    for h, reqs in ((h1, b1), (h2, b2)):
        for r, Y in zip(reqs, ex.finish(h)):
            alone = sg.spgemm("or_and_bool", dA, r.X).to_host()
            Yh = Y.to_host()
            assert np.array_equal(Yh.ptr, alone.ptr) and np.array_equal(Yh.idx, alone.idx)


@pytest.mark.gpu
def test_gpu_frontier_servers_match_oracle():
    """Requests arriving as host frontier triples (one source per column, or a
    source's neighbourhood: several entries per column, repeated sources across
    columns): the batched server (operands built on the device, one product per
    batch) and the FIFO server both return, per request, exactly the oracle's
    A X_r."""
    import torch
    import oracle
    import paper_1006_2183_amd as sg
    from paper_1006_2183_amd.serve import Frontier, FrontierBatchExecutor, FrontierFifoExecutor
    from tests.helpers import assert_same
    sg.load_library()
    A = W.rmat_matrix(13, 16, "or_and_bool", "csc", seed=3)
    dA = sg.DevMat.from_host(A, "cuda", "or_and_bool")
    colcount = np.diff(A.ptr)
    rng = np.random.default_rng(8)
    fronts = []
    for i in range(40):
        k = int(rng.integers(1, 130))
        if i % 2:
            fronts.append(Frontier.sources(rng.integers(0, A.nrows, k)))
        else:
            X = W.bfs_frontier(A.nrows, k, seed=500 + i, A=A, depth=1)
            r, c, _ = X.triples()
            fronts.append(Frontier(r.astype(np.int32), c.astype(np.int32), k))
    arr = W.poisson_arrivals(20000.0, len(fronts), 3)
    for ex, mb in ((FrontierBatchExecutor(dA), 16), (FrontierFifoExecutor(dA), 1)):
        reqs = [Request(i, float(arr[i]), f, frontier_bound(colcount, f)) for i, f in enumerate(fronts)]
        done = Scheduler(ex, pool_entries=1 << 24, max_batch=mb, max_inflight=2 if mb > 1 else 1).run(reqs)
        assert len(done) == len(reqs)
        torch.cuda.synchronize()
        assert all(r.status == "done" for r in done)
        for r in done:
            Y = (r.result[0] if isinstance(r.result, list) else r.result).to_host()
            f = fronts[r.rid]
            X = W.from_triples(f.rows, f.cols, None, A.nrows, f.k, "csc", "or_and_bool")
            R, _ = oracle.spgemm("or_and_bool", A, X)
            assert_same(Y, R, "or_and_bool", what=f"request {r.rid}")
