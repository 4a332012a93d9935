"""GPU parity at the measured sizes, in the launch forms the benchmark times: the
scale-24 SUMMA share (fused persistent launch, partials then merge, graph
replay; the whole output against the oracle on the matching strips), the
largest Galerkin instances (exact closed form) and the scale-20 served
expansions (exact closed form for every column)."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import assert_same

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1006_2183_amd as sg
    sg.load_library()
    return sg


def _strips(a_blocks, b_blocks, grid, b, sr):
    """Host CSC of the strips A(I, :) (b x grid*b) and A(:, J) (grid*b x b) that the
    stage blocks cut (input preparation for the oracle: C_IJ = A(I, :) A(:, J),
    the block identity of Section 3.2)."""
    ra, ca, va, rb, cb, vb = [], [], [], [], [], []
    for k in range(grid):
        A, B = a_blocks[k], b_blocks[k]
        ra.append(A.idx.astype(np.int64)); va.append(A.val)
        ca.append(np.repeat(A.vid.astype(np.int64), np.diff(A.ptr)) + k * b)
        rb.append(B.idx.astype(np.int64) + k * b); vb.append(B.val)
        cb.append(np.repeat(B.vid.astype(np.int64), np.diff(B.ptr)))
    SA = W.from_triples(np.concatenate(ra), np.concatenate(ca), np.concatenate(va), b, grid * b, "csc", sr)
    SB = W.from_triples(np.concatenate(rb), np.concatenate(cb), np.concatenate(vb), grid * b, b, "csc", sr)
    return SA, SB


def _assert_whole(C, R, what):
    """Every column of the DCSC result C against the oracle's CSC result R: the same
    stored columns (empty ones elided), ids bit-exact, values within 1e-12 relative."""
    lens = np.diff(R.ptr)
    nz = np.flatnonzero(lens)
    assert np.array_equal(C.vid.astype(np.int64), nz), f"{what}: stored columns differ"
    assert np.array_equal(np.diff(C.ptr), lens[nz]), f"{what}: column sizes differ"
    assert np.array_equal(C.idx, R.idx), f"{what}: row ids differ"
    err = np.abs(C.val - R.val)
    bad = err > 1e-12 * np.abs(R.val)
    assert not bad.any(), f"{what}: {int(bad.sum())} values beyond 1e-12"


def test_summa_share_scale24_whole_output(sg):
    """The whole scale-24 SUMMA share (process (0,0) of a 64 x 64 grid), in the three
    forms the benchmark times (fused persistent launch, 64 partials then a 64-way
    merge, graph replay of a plan with entry records), against the oracle's product
    of the strips, column by column."""
    import torch
    from paper_1006_2183_amd import batched as BT
    sr, scale, grid = "plus_times_f64", 24, 64
    _say("case SUMMA share scale 24, 64 stages: generating")
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (0, 0), semiring=sr, seed=24, device="cuda", fmt="dcsc")
    b = (1 << scale) // grid
    dA = [sg.DevMat.from_host(x, "cuda", sr) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", sr) for x in b_blocks]
    _say("case SUMMA share scale 24: oracle on the strips")
    SA, SB = _strips(a_blocks, b_blocks, grid, b, sr)
    R, flops = oracle.spgemm_threads(sr, SA, SB)
    _say(f"case SUMMA share scale 24: oracle done ({flops} multiplications, {R.nnz} entries); fused launch")
    C = BT.summa_share(sr, dA, dB, batched=True).to_host()
    _assert_whole(C, R, "fused")
    _say("case SUMMA share scale 24: partials then merge")
    parts = [sg.spgemm(sr, x, y, out_fmt="dcsc") for x, y in zip(dA, dB)]
    C = BT.merge_partials(sr, parts).to_host()
    del parts
    _assert_whole(C, R, "partials+merge")
    _say("case SUMMA share scale 24: graph replay with entry records")
    plan = BT.summa_share_plan(sr, dA, dB, tuning=sg.make_tuning(sr, entry_mb=1024))
    assert plan.infos[0]["flops"] == flops
    G = BT.GraphedNumeric(plan)
    for rep in range(2):
        G.replay()
        torch.cuda.synchronize()
        _assert_whole(G.outputs[0].to_host(), R, f"graph replay {rep}")
    plan.destroy()


@pytest.mark.parametrize("n", [128, 96])
def test_galerkin_full_size_closed_form(sg, n):
    from paper_1006_2183_amd import batched as BT
    _say(f"case Galerkin n={n}")
    L = W.laplacian_7pt(n, "csr")
    P = W.aggregation_p(n, "csr")
    R = W.transpose(P, "csr")
    dev = lambda M: sg.DevMat.from_host(M, "cuda")
    out = BT.galerkin_rap("plus_times_f64", [dev(R), dev(R)], [dev(L), dev(L)], [dev(P), dev(P)], batched=True)
    Lc = W.laplacian_7pt(n // 2, "csr")
    Lc.val = Lc.val * 4.0
    for o in out:
        assert_same(o.to_host(), Lc, "plus_times_f64", 0.0, f"n={n}")


def test_serving_scale20_closed_form(sg):
    import torch
    from paper_1006_2183_amd import serve as SV
    sr = "or_and_bool"
    _say("case served expansions, R-MAT scale 20")
    A = W.rmat_matrix(20, 16, sr, "csc", seed=1, device="cuda")
    dA = sg.DevMat.from_host(A, "cuda", sr)
    colcount = np.diff(A.ptr)
    rng = np.random.default_rng(101)
    reqs, srcs = [], []
    arr = W.poisson_arrivals(4000.0, 80, 7)
    for i in range(80):
        X = W.bfs_frontier(A.nrows, int(rng.integers(1, 513)), seed=2000 + i)
        srcs.append(X.idx.astype(np.int64))
        reqs.append(SV.Request(i, float(arr[i]), sg.DevMat.from_host(X, "cuda", sr), SV.frontier_bound(colcount, X)))
    done = SV.Scheduler(SV.GpuBatchExecutor(sr, dA), 1 << 26, max_batch=64, max_inflight=2).run(reqs)
    torch.cuda.synchronize()
    assert all(r.status == "done" for r in done)
    for r in done:
        Y = r.result.to_host()
        for s_, u in enumerate(srcs[r.rid]):
            assert np.array_equal(Y.idx[Y.ptr[s_]:Y.ptr[s_ + 1]], A.idx[A.ptr[u]:A.ptr[u + 1]]), \
                f"request {r.rid} column {s_}"
