"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Integer and boolean results must match bit for bit, patterns always; FP64
(+,*) values within 1e-12 relative per entry; FP32 (+,*) within
2 * d * 2^-24 relative, d being the number of terms of the entry (each side
sums the same positive terms in a different order, and the recursive-sum
bound of one side is (d - 1) u).
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import assert_canonical, assert_same, triples

pytestmark = pytest.mark.gpu

SEMIRINGS = ["plus_times_f64", "plus_times_f32", "min_plus_i32", "or_and_bool"]


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


def term_counts(A, B):
    """Number of products per output entry (oracle on all-ones operands)."""
    def ones(M):
        import types
        return types.SimpleNamespace(fmt=M.fmt, nrows=M.nrows, ncols=M.ncols, ptr=M.ptr, idx=M.idx,
                                     vid=M.vid, val=np.ones(M.nnz))
    C, _ = oracle.spgemm("plus_times_f64", ones(A), ones(B))
    return C


def check(semiring, Cg, A, B, what=""):
    R, flops = oracle.spgemm(semiring, A, B)
    assert_canonical(Cg)
    if semiring == "plus_times_f32":
        assert_same(Cg, R, "or_and_bool", what=what)
        _, _, vg = triples(Cg)
        _, _, vr = triples(R)
        _, _, d = triples(term_counts(A, B))
        err = np.abs(vg.astype(np.float64) - vr.astype(np.float64))
        tol = 2.0 * d * 2.0 ** -24 * np.abs(vr.astype(np.float64))
        assert np.all(err <= tol), f"{what}: f32 values beyond 2 d u"
    else:
        assert_same(Cg, R, semiring, 1e-12, what)
    return R, flops


def gpu_product(sg, semiring, A, B, out_fmt=None, batched=False, **tune):
    dA = sg.DevMat.from_host(A, "cuda", semiring)
    dB = sg.DevMat.from_host(B, "cuda", semiring)
    t = sg.make_tuning(semiring, **tune) if tune else None
    plan = sg.spgemm_symbolic(semiring, [dA], [dB], out_fmt=out_fmt, tuning=t)
    C = plan.alloc_outputs()
    (sg.spgemm_batched if batched else sg.spgemm_numeric)(plan, C)
    import torch
    torch.cuda.synchronize()
    info = plan.infos[0]
    plan.destroy()
    return C[0].to_host(), info


@pytest.mark.parametrize("semiring", SEMIRINGS)
@pytest.mark.parametrize("batched", [False, True])
def test_rmat_s10_default_tiers(sg, semiring, batched):
    _say(f"case rmat s10 ef8 {semiring} batched={batched}")
    A = W.rmat_matrix(10, 8, semiring, "csr", seed=1)
    C, info = gpu_product(sg, semiring, A, A, batched=batched)
    R, flops = check(semiring, C, A, A, "rmat10")
    assert info["flops"] == flops
    assert info["nnz"] == R.nnz
    assert info["nnz_ub"] >= R.nnz


@pytest.mark.parametrize("semiring", SEMIRINGS)
@pytest.mark.parametrize("force,mid_kind,heavy_kind,bitmap_mb", [(0, 0, 0, 4096), (1, 0, 0, 4096), (1, 1, 0, 4096),
                                                                 (2, 0, 0, 4096), (2, 0, 0, 0), (2, 0, 0, 1),
                                                                 (2, 0, 1, 4096), (-1, 0, 0, 4096), (-1, 1, 1, 0),
                                                                 (3, 0, 0, 4096)])
def test_forced_tiers_several_windows(sg, semiring, force, mid_kind, heavy_kind, bitmap_mb):
    """Every tier on every vector it can take. 16 KB of LDS: a rank window's words and values
    share 2048 (f64) or 4096 (4-byte values) value slots over 1K/2K-id buckets, so heavy rows
    split into several planned windows; dense windows are ~2K ids wide over 8192 columns (the
    last partial).
    bitmap_mb 0 re-marks every window; 1 MiB keeps the bitmaps of only part of the heavy vectors."""
    _say(f"case forced tier {force} mid_kind {mid_kind} heavy_kind {heavy_kind} bitmap_mb {bitmap_mb} {semiring}")
    A = W.rmat_matrix(13, 8, semiring, "csr", seed=4)
    C, info = gpu_product(sg, semiring, A, A, force_tier=force, mid_kind=mid_kind, heavy_kind=heavy_kind,
                          lds_bytes=16384, block_threads=256, bitmap_mb=bitmap_mb,
                          heavy_lds_bytes=16384, heavy_threads=256)
    check(semiring, C, A, A, f"force{force}")
    if force == 2:
        assert info["n_mid"] == 0 and info["n_tiny"] == 0
    if force == 1:
        assert info["n_mid"] > 0
    if force == 3:
        assert info["n_small"] > 0


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32", "or_and_bool"])
@pytest.mark.parametrize("fa,fb,fo", [("csc", "csc", "csc"), ("dcsc", "dcsc", "dcsc"), ("dcsr", "dcsr", "dcsr"),
                                      ("csr", "dcsr", "csr"), ("dcsc", "csc", "dcsc"), ("csr", "csr", "dcsr"),
                                      ("csc", "dcsc", "dcsc")])
def test_formats(sg, semiring, fa, fb, fo):
    _say(f"case formats {fa} {fb} -> {fo} {semiring}")
    A = W.rmat_matrix(11, 8, semiring, "csr", seed=6)
    Af = W.to_format(A, fa, semiring)
    Bf = W.to_format(A, fb, semiring)
    for force in (-1, 2):
        C, _ = gpu_product(sg, semiring, Af, Bf, out_fmt=fo, force_tier=force, lds_bytes=8192, block_threads=128,
                                heavy_lds_bytes=8192, heavy_threads=128)
        assert C.fmt == fo
        check(semiring, C, Af, Bf, f"{fa}{fb}{fo}")


@pytest.mark.parametrize("fmt", ["csc", "dcsc", "csr", "dcsr"])
def test_paper_fig8_example_gpu(sg, fmt):
    from tests.golden import fixtures
    f = fixtures.read("fig8_example.txt")
    a = np.array(f["A"], dtype=np.int64) - 1
    b = np.array(f["B"], dtype=np.int64) - 1
    A = W.from_triples(a[:, 0], a[:, 1], np.ones(len(a)), 6, 6, fmt)
    B = W.from_triples(b[:, 0], b[:, 1], np.ones(len(b)), 6, 6, fmt)
    for force in (-1, 1, 2):
        C, info = gpu_product(sg, "plus_times_f64", A, B, force_tier=force)
        assert info["flops"] == 19
        exp = np.array(f["C"], dtype=np.int64)
        R = W.from_triples(exp[:, 0] - 1, exp[:, 1] - 1, exp[:, 2].astype(np.float64), 6, 6, "csr")
        assert_same(C, R, "plus_times_f64", 0.0)


def test_aux_matches_paper_example(sg):
    from tests.golden import fixtures
    f = fixtures.read("dcsc_example.txt")
    n = int(f["n"][0][0])
    t = f["triples"]
    r = np.array([int(x[0]) for x in t]) - 1
    c = np.array([int(x[1]) for x in t]) - 1
    d = W.from_triples(r, c, np.array([float(x[2]) for x in t]), n, n, "dcsc")
    aux = sg.build_aux(sg.DevMat.from_host(d, "cuda")).cpu().numpy()
    assert (aux + 1).tolist() == [int(x) for x in f["aux"][0]]


@pytest.mark.parametrize("semiring", SEMIRINGS)
def test_edge_cases(sg, semiring):
    _say(f"case edge {semiring}")
    rng = np.random.default_rng(0)
    for fmt in ("csr", "dcsc"):
        # 1 x 1
        X = W.from_triples([0], [0], W.random_values(rng, 1, semiring), 1, 1, fmt, semiring)
        C, _ = gpu_product(sg, semiring, X, X)
        check(semiring, C, X, X, "1x1")
        # an operand with no entries
        E = W.random_sparse(40, 30, 0.0, semiring, fmt, 1)
        B = W.random_sparse(30, 20, 0.3, semiring, fmt, 2)
        C, info = gpu_product(sg, semiring, E, B)
        assert info["nnz"] == 0 and info["flops"] == 0
        check(semiring, C, E, B, "empty")
        # one dense column of B against a hub: a single heavy output vector
        n = 3000
        col = np.arange(n)
        Bd = W.from_triples(col, np.zeros(n, dtype=np.int64), W.random_values(rng, n, semiring), n, 1, fmt, semiring)
        Ah = W.random_sparse(n, n, 0.004, semiring, fmt, 3)
        C, info = gpu_product(sg, semiring, Ah, Bd, lds_bytes=4096, block_threads=64,
                                  heavy_lds_bytes=4096, heavy_threads=64)
        check(semiring, C, Ah, Bd, "dense column")
        # rectangular, mostly empty vectors
        A = W.random_sparse(500, 7, 0.05, semiring, fmt, 4)
        B = W.random_sparse(7, 900, 0.01, semiring, fmt, 5)
        C, _ = gpu_product(sg, semiring, A, B)
        check(semiring, C, A, B, "rect")


def test_identity_and_permutation_bit_exact(sg):
    for semiring in ("plus_times_f64", "min_plus_i32"):
        A = W.rmat_matrix(12, 8, semiring, "csr", seed=8)
        n = A.nrows
        Q = W.permutation_matrix(n, 5, "csr", semiring)
        for L, R in ((A, Q), (Q, A), (A, W.identity_matrix(n, "csr", semiring))):
            C, _ = gpu_product(sg, semiring, L, R)
            Ro, _ = oracle.spgemm(semiring, L, R)
            assert_same(C, Ro, semiring, 0.0)


def test_errors(sg):
    import torch
    A = W.rmat_matrix(8, 8, "plus_times_f64", "csr", seed=2)
    dA = sg.DevMat.from_host(A, "cuda")
    plan = sg.spgemm_symbolic("plus_times_f64", [dA], [dA])
    C = plan.alloc_outputs()[0]
    C.idx = C.idx[: max(0, C.idx.numel() - 1)]
    with pytest.raises(sg.SgError) as e:
        sg.spgemm_numeric(plan, [C])
    assert e.value.status == -6
    plan.destroy()
    # a non-canonical operand is reported by validation
    bad = sg.DevMat.from_host(A, "cuda")
    idx = bad.idx.clone()
    a, b = int(A.ptr[3]), int(A.ptr[4])
    if b - a >= 2:
        idx[a], idx[a + 1] = bad.idx[a + 1], bad.idx[a]
    else:
        idx[0] = A.ncols + 5
    bad.idx = idx
    assert sg.validate(dA)
    assert not sg.validate(bad)
    t = sg.make_tuning("plus_times_f64", validate=1)
    with pytest.raises(sg.SgError) as e:
        sg.spgemm_symbolic("plus_times_f64", [bad], [dA], tuning=t)
    assert e.value.status == -3
    torch.cuda.synchronize()


def _row_block(A, r0, r1):
    """Host CSR of rows [r0, r1) of A (input preparation for the oracle)."""
    import types
    a, b = int(A.ptr[r0]), int(A.ptr[r1])
    return types.SimpleNamespace(fmt="csr", nrows=r1 - r0, ncols=A.ncols, ptr=A.ptr[r0:r1 + 1] - a,
                                 idx=A.idx[a:b], val=None if A.val is None else A.val[a:b], vid=None)


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32"])
def test_rmat_s18_whole_output(sg, semiring):
    """The full-size product (R-MAT scale 18, edge factor 16) in the benchmark's
    configuration, compared with the oracle on EVERY row: row blocks of C = A A
    against the oracle's A(rows, :) A (row i of C is the paper's column-wise
    product on the transposes), ids bit-exact, values within 1e-12 (FP64) or
    exact (min-plus)."""
    import torch
    _say(f"case rmat s18 ef16 {semiring}")
    A = W.rmat_matrix(18, 16, semiring, "csr", seed=1)
    dA = sg.DevMat.from_host(A, "cuda", semiring)
    plan = sg.spgemm_symbolic(semiring, [dA], [dA])
    info = plan.infos[0]
    Cd = plan.alloc_outputs()[0]
    sg.spgemm_numeric(plan, [Cd])
    torch.cuda.synchronize()
    plan.destroy()
    # flops identity (Section 2.4): sum over k of nnz(A(:,k)) nnz(A(k,:))
    colc = np.bincount(A.idx, minlength=A.ncols).astype(np.int64)
    rowc = np.diff(A.ptr).astype(np.int64)
    assert info["flops"] == int(np.dot(colc, rowc))
    cptr = Cd.ptr.cpu().numpy()
    assert cptr[0] == 0 and np.all(np.diff(cptr) >= 0)
    assert info["nnz"] == cptr[-1] and info["nnz"] <= info["flops"]
    n = A.nrows
    nblk = 16
    # row blocks of about equal work (flops per row = sum of the lengths of the rows it gathers)
    rf = np.zeros(n, dtype=np.int64)
    np.add.at(rf, np.repeat(np.arange(n), np.diff(A.ptr)), rowc[A.idx])
    edges = np.searchsorted(np.cumsum(rf), np.linspace(0, rf.sum(), nblk + 1)[1:-1])
    bounds = [0] + sorted(set(int(e) for e in edges if 0 < e < n)) + [n]
    tot = 0
    for r0, r1 in zip(bounds[:-1], bounds[1:]):
        R, f = oracle.spgemm_threads(semiring, _row_block(A, r0, r1), A)
        tot += f
        a, b = int(cptr[r0]), int(cptr[r1])
        assert np.array_equal(cptr[r0:r1 + 1] - a, R.ptr), f"rows [{r0}, {r1}): sizes differ"
        assert np.array_equal(Cd.idx[a:b].cpu().numpy(), R.idx), f"rows [{r0}, {r1}): column ids differ"
        cval = Cd.val[a:b].cpu().numpy()
        if semiring == "min_plus_i32":
            assert np.array_equal(cval, R.val), f"rows [{r0}, {r1}): values differ"
        else:
            bad = np.abs(cval - R.val) > 1e-12 * np.abs(R.val)
            assert not bad.any(), f"rows [{r0}, {r1}): {int(bad.sum())} values beyond 1e-12"
        _say(f"  rows [{r0}, {r1}) ok")
    assert tot == info["flops"]


@pytest.mark.parametrize("entry_mb", [0, 1, 2048])
def test_entry_records_budget(sg, entry_mb):
    """Heavy windows with entry records (all, some within a 1 MiB budget, none) equal the oracle."""
    semiring = "min_plus_i32"
    A = W.rmat_matrix(12, 16, semiring, "csr", seed=21)
    _say(f"case entry records entry_mb={entry_mb}")
    C, info = gpu_product(sg, semiring, A, A, lds_bytes=8192, block_threads=256, heavy_lds_bytes=8192,
                          heavy_threads=256, entry_mb=entry_mb)
    assert info["n_heavy_items"] > info["n_heavy"] > 0  # several windows per heavy vector
    check(semiring, C, A, A, f"entry_mb={entry_mb}")
