"""GPU parity of the fused chain product C = X Y Z (the intermediate never
written; the triple products of multigrid setup named in the paper's Section
8) against the two-call oracle X (Y Z) / (X Y) Z and the Galerkin closed form
R L_n P = 4 L_{n/2}, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import assert_canonical, assert_same

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


def _two_call(semiring, X, Y, Z):
    if X.fmt in ("csc", "dcsc"):
        YZ, _ = oracle.spgemm(semiring, Y, Z)
        return oracle.spgemm(semiring, X, YZ)[0]
    XY, _ = oracle.spgemm(semiring, X, Y)
    return oracle.spgemm(semiring, XY, Z)[0]


def _fused(sg, semiring, Xs, Ys, Zs, batched=True, check=False, **tune):
    import torch
    dev = lambda M: sg.DevMat.from_host(M, "cuda", semiring)
    dX, dY, dZ = [dev(x) for x in Xs], [dev(y) for y in Ys], [dev(z) for z in Zs]
    t = sg.make_tuning(semiring, **tune) if tune else None
    plan = sg.chain_symbolic(semiring, dX, dY, dZ, tuning=t)
    C = plan.alloc_outputs()
    (sg.spgemm_batched if batched else sg.spgemm_numeric)(plan, C)
    torch.cuda.synchronize()
    if check:
        lds, cnt = plan.check()
        assert lds == 0 and cnt == 0, (lds, cnt)
    infos = plan.infos
    plan.destroy()
    return [c.to_host() for c in C], infos


@pytest.mark.parametrize("fmt", ["csr", "csc"])
def test_galerkin_closed_form_every_size(sg, fmt):
    """R L_n P = 4 L_{n/2} exactly (FP64), for every grid size of the workload, all
    instances in one fused plan."""
    sizes = [32, 48, 64, 96, 128]
    _say(f"case fused Galerkin {fmt}")
    Ls = [W.to_format(W.laplacian_7pt(n, "csr"), fmt) for n in sizes]
    Ps = [W.to_format(W.aggregation_p(n, "csr"), fmt) for n in sizes]
    Rs = [W.transpose(P, fmt) for P in Ps]
    for batched in (True, False):
        C, infos = _fused(sg, "plus_times_f64", Rs, Ls, Ps, batched=batched)
        for i, n in enumerate(sizes):
            Lc = W.to_format(W.laplacian_7pt(n // 2, "csr"), fmt)
            Lc.val = Lc.val * 4.0
            assert_canonical(C[i])
            assert_same(C[i], Lc, "plus_times_f64", 0.0, f"n={n}")
            assert infos[i]["nnz"] == Lc.nnz
    # and the two-call oracle on one size
    R2 = _two_call("plus_times_f64", Rs[0], Ls[0], Ps[0])
    assert_same(C[0], R2, "plus_times_f64", 0.0, "two-call")


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32", "or_and_bool"])
@pytest.mark.parametrize("fmt", ["csr", "csc"])
@pytest.mark.parametrize("force", [-1, 1])
def test_random_chains_match_two_call_oracle(sg, semiring, fmt, force):
    """Uneven random chains (R-MAT middle operands, random rectangular outer ones)
    with vectors in both fused tiers, against the two-call oracle."""
    _say(f"case chains {semiring} {fmt} force={force}")
    Xs, Ys, Zs = [], [], []
    for i, (m, k, l, n) in enumerate([(300, 1024, 1024, 200), (64, 256, 256, 700), (1000, 512, 512, 9)]):
        scale = int(np.log2(k))
        Xs.append(W.to_format(W.random_sparse(m, k, 0.004, semiring, "csr", 10 + i), fmt, semiring))
        Ys.append(W.to_format(W.rmat_matrix(scale, 4, semiring, "csr", seed=20 + i), fmt, semiring))
        Zs.append(W.to_format(W.random_sparse(l, n, 0.006, semiring, "csr", 30 + i), fmt, semiring))
    C, infos = _fused(sg, semiring, Xs, Ys, Zs, force_tier=force, check=False)
    for i in range(len(Xs)):
        R = _two_call(semiring, Xs[i], Ys[i], Zs[i])
        assert_canonical(C[i])
        assert_same(C[i], R, semiring, 1e-12, f"chain {i}")
    if force == 1:
        assert infos[0]["n_mid"] > 0


def test_chain_invariants_and_value_reuse(sg):
    """The checking build (LDS back to zero after every mid vector, counts equal),
    then a repeated setup: new values, same structure, the same plan's numeric
    phase (plain, and replayed from a graph)."""
    import torch
    from paper_1006_2183_amd import binding
    from paper_1006_2183_amd import batched as BT
    sr = "plus_times_f64"
    _say("case chain invariants and reuse")
    Xh = W.random_sparse(400, 2048, 0.003, sr, "csc", 1)
    Yh = W.rmat_matrix(11, 8, sr, "csc", seed=2)
    Zh = W.random_sparse(2048, 300, 0.004, sr, "csc", 3)
    prev = binding.use_library(binding.CHECK_LIB_PATH)
    try:
        for force in (-1, 1):
            (C,), _ = _fused(sg, sr, [Xh], [Yh], [Zh], check=True, force_tier=force)
            assert_same(C, _two_call(sr, Xh, Yh, Zh), sr, 1e-12, f"check force={force}")
    finally:
        binding.use_library(prev)
    dX, dY, dZ = (sg.DevMat.from_host(M, "cuda", sr) for M in (Xh, Yh, Zh))
    plan = BT.galerkin_chain_plan(sr, [dX], [dY], [dZ])
    G = BT.GraphedNumeric(plan)
    for rep, scale in enumerate((1.0, 3.0, 0.5)):
        dY.val.copy_(torch.as_tensor(Yh.val * scale).cuda())
        Y2 = W.SpMat(Yh.fmt, Yh.nrows, Yh.ncols, Yh.ptr, Yh.idx, Yh.val * scale)
        R = _two_call(sr, Xh, Y2, Zh)
        G.replay()
        torch.cuda.synchronize()
        assert_same(G.outputs[0].to_host(), R, sr, 1e-12, f"graph replay {rep}")
        (C,) = plan.alloc_outputs()
        sg.spgemm_numeric(plan, [C])
        torch.cuda.synchronize()
        assert_same(C.to_host(), R, sr, 1e-12, f"numeric {rep}")
    plan.destroy()


def test_chain_beyond_fused_tiers_is_refused(sg):
    sr = "plus_times_f64"
    X = W.random_sparse(50, 400, 0.5, sr, "csr", 5)
    Y = W.random_sparse(400, 400, 0.5, sr, "csr", 6)
    Z = W.random_sparse(400, 60, 0.5, sr, "csr", 7)
    dev = lambda M: sg.DevMat.from_host(M, "cuda", sr)
    with pytest.raises(sg.SgError) as e:
        sg.chain_symbolic(sr, [dev(X)], [dev(Y)], [dev(Z)], tuning=sg.make_tuning(sr, lds_bytes=4096))
    assert e.value.status == -4
