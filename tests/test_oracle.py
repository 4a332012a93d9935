"""Pins for the CPU oracle: what the paper and the mathematics fix, not the oracle itself.

Each test checks the oracle against something independent of its Gustavson
loop: the inner-product definition evaluated by brute force (Eq. 1), the
paper's worked example (Figures 8-9), a library sparse product (scipy) for
the ordinary (+,*) and boolean cases, closed forms (identity, permutation,
Galerkin coarsening of the 7-point grid), the flops identity and the size
bound of Section 2.4, and the block identity behind Sparse SUMMA (Section 3.2).
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W
from tests.golden import fixtures
from tests.helpers import INT32_MAX, assert_canonical, assert_same, triples

SEMIRINGS = ["plus_times_f64", "plus_times_f32", "min_plus_i32", "or_and_bool"]
FMT_PAIRS = [("csr", "csr"), ("csc", "csc"), ("dcsr", "dcsr"), ("dcsc", "dcsc"),
             ("csr", "dcsr"), ("dcsc", "csc")]


def _sat(a, b):
    if a == INT32_MAX or b == INT32_MAX:
        return INT32_MAX
    return max(min(int(a) + int(b), INT32_MAX), -INT32_MAX - 1)


def brute_force(semiring, A, B):
    """Eq. 1: C(i,j) = (+)_l A(i,l) (x) B(l,j) over every (i, j), ascending l."""
    ra, ca, va = triples(A)
    rb, cb, vb = triples(B)
    da = {}
    db = {}
    for q in range(ra.size):
        da[(int(ra[q]), int(ca[q]))] = None if va is None else va[q]
    for q in range(rb.size):
        db[(int(rb[q]), int(cb[q]))] = None if vb is None else vb[q]
    rows, cols, vals = [], [], []
    for i in range(A.nrows):
        for j in range(B.ncols):
            acc = None
            hit = False
            for l in range(A.ncols):
                if (i, l) in da and (l, j) in db:
                    a, b = da[(i, l)], db[(l, j)]
                    if semiring == "plus_times_f64":
                        t = float(a) * float(b)
                        acc = t if not hit else acc + t
                    elif semiring == "plus_times_f32":
                        t = np.float32(a) * np.float32(b)
                        acc = t if not hit else np.float32(acc + t)
                    elif semiring == "min_plus_i32":
                        t = _sat(a, b)
                        acc = t if not hit else min(acc, t)
                    hit = True
            if hit:
                rows.append(i)
                cols.append(j)
                vals.append(acc)
    vdt = W.VALUE_DTYPES[semiring]
    v = None if vdt is None else np.array(vals, dtype=vdt)
    return W.from_triples(np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64), v,
                          A.nrows, B.ncols, "csr", semiring)


def _rand(m, n, density, semiring, fmt, seed, big=False):
    M = W.random_sparse(m, n, density, semiring, fmt, seed)
    if big and semiring == "min_plus_i32" and M.nnz:
        rng = np.random.default_rng(seed + 99)
        M.val = rng.integers(2 ** 30, INT32_MAX, size=M.nnz, dtype=np.int32)
    return M


@pytest.mark.parametrize("semiring", SEMIRINGS)
@pytest.mark.parametrize("fa,fb", FMT_PAIRS)
def test_bruteforce_tiny(semiring, fa, fb):
    if (fa in ("csr", "dcsr")) != (fb in ("csr", "dcsr")):
        pytest.skip("mixed orientation")
    rng = np.random.default_rng(1234)
    for trial in range(12):
        m, k, n = (int(x) for x in rng.integers(1, 13, size=3))
        dens = [0.05, 0.2, 0.6][trial % 3]
        A = _rand(m, k, dens, semiring, fa, 10 * trial + 1, big=trial % 4 == 3)
        B = _rand(k, n, dens, semiring, fb, 10 * trial + 2, big=trial % 4 == 3)
        C, flops = oracle.spgemm(semiring, A, B)
        assert_canonical(C)
        R = brute_force(semiring, A, B)
        # ascending-l fold on both sides: bit-identical, floating point included
        assert_same(C, R, semiring, 0.0, f"trial {trial}")


def test_min_plus_saturates():
    # entries near INT32_MAX: the (x) of (min,+) saturates at +infinity
    A = W.from_triples([0, 0], [0, 1], np.array([2 ** 31 - 10, 5], np.int32), 1, 2, "csr", "min_plus_i32")
    B = W.from_triples([0, 1], [0, 0], np.array([100, 7], np.int32), 2, 1, "csr", "min_plus_i32")
    C, flops = oracle.spgemm("min_plus_i32", A, B)
    assert flops == 2
    assert C.val.tolist() == [12]
    A.val = np.array([2 ** 31 - 2, 2 ** 31 - 3], np.int32)
    C, _ = oracle.spgemm("min_plus_i32", A, B)
    assert C.val.tolist() == [INT32_MAX]


def _fig8():
    f = fixtures.read("fig8_example.txt")
    a = np.array(f["A"], dtype=np.int64) - 1
    b = np.array(f["B"], dtype=np.int64) - 1
    return f, a, b


@pytest.mark.parametrize("fmt", ["csc", "dcsc", "csr", "dcsr"])
def test_paper_fig8_example(fmt):
    f, a, b = _fig8()
    A = W.from_triples(a[:, 0], a[:, 1], np.ones(len(a)), 6, 6, fmt)
    B = W.from_triples(b[:, 0], b[:, 1], np.ones(len(b)), 6, 6, fmt)
    if fmt == "dcsc":
        assert (A.vid + 1).tolist() == [int(x) for x in f["ajc"][0]]
        Bt = W.transpose(B, "dcsc")
        assert (Bt.vid + 1).tolist() == [int(x) for x in f["btjc"][0]]
        isect = sorted(set(A.vid.tolist()) & set(Bt.vid.tolist()))
        assert [x + 1 for x in isect] == [int(x) for x in f["isect"][0]]
    C, flops = oracle.spgemm("plus_times_f64", A, B)
    assert flops == int(f["flops"][0][0])
    exp = np.array(f["C"], dtype=np.int64)
    R = W.from_triples(exp[:, 0] - 1, exp[:, 1] - 1, exp[:, 2].astype(np.float64), 6, 6, "csr")
    assert C.nnz == 13
    assert_same(C, R, "plus_times_f64", 0.0)
    # boolean semiring gives the same pattern
    Ab = W.from_triples(a[:, 0], a[:, 1], None, 6, 6, fmt, "or_and_bool")
    Bb = W.from_triples(b[:, 0], b[:, 1], None, 6, 6, fmt, "or_and_bool")
    Cb, fb = oracle.spgemm("or_and_bool", Ab, Bb)
    assert fb == 19
    assert_same(Cb, R, "or_and_bool")


def test_paper_dcsc_encoding():
    f = fixtures.read("dcsc_example.txt")
    n = int(f["n"][0][0])
    t = f["triples"]
    r = np.array([int(x[0]) for x in t]) - 1
    c = np.array([int(x[1]) for x in t]) - 1
    v = np.array([float(x[2]) for x in t])
    csc = W.from_triples(r, c, v, n, n, "csc")
    assert (csc.ptr + 1).tolist() == [int(x) for x in f["csc_jc"][0]]
    assert (csc.idx + 1).tolist() == [int(x) for x in f["ir"][0]]
    assert csc.val.tolist() == [float(x) for x in f["num"][0]]
    d = W.from_triples(r, c, v, n, n, "dcsc")
    assert (d.vid + 1).tolist() == [int(x) for x in f["dcsc_jc"][0]]
    assert (d.ptr + 1).tolist() == [int(x) for x in f["dcsc_cp"][0]]
    # a product through the doubly compressed form equals the plain one
    I = W.identity_matrix(n, "dcsc")
    C, flops = oracle.spgemm("plus_times_f64", d, I)
    assert flops == 4
    assert_same(C, d, "plus_times_f64", 0.0)


def _to_scipy(M):
    r, c, v = triples(M)
    data = np.ones(r.size) if v is None else v.astype(np.float64)
    return sp.csr_matrix((data, (r, c)), shape=(M.nrows, M.ncols))


@pytest.mark.parametrize("fmt", ["csr", "csc", "dcsc"])
def test_scipy_plus_times(fmt):
    A = W.random_sparse(300, 400, 0.02, "plus_times_f64", fmt, 5)
    B = W.random_sparse(400, 250, 0.03, "plus_times_f64", fmt, 6)
    C, flops = oracle.spgemm("plus_times_f64", A, B)
    S = (_to_scipy(A) @ _to_scipy(B)).tocsr()
    S.sort_indices()
    r = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
    R = W.from_triples(r, S.indices, S.data, S.shape[0], S.shape[1], "csr")
    assert_same(C, R, "plus_times_f64", 1e-13)


def test_scipy_rmat_plus_times_and_bool():
    A = W.rmat_matrix(9, 8, "plus_times_f64", "csr", seed=3)
    C, flops = oracle.spgemm("plus_times_f64", A, A)
    S = (_to_scipy(A) @ _to_scipy(A)).tocsr()
    S.sort_indices()
    r = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
    R = W.from_triples(r, S.indices, S.data, S.shape[0], S.shape[1], "csr")
    assert_same(C, R, "plus_times_f64", 1e-12)
    Ab = W.rmat_matrix(9, 8, "or_and_bool", "csc", seed=3)
    Cb, fb = oracle.spgemm("or_and_bool", Ab, Ab)
    assert fb == flops
    assert_same(Cb, R, "or_and_bool")


def _flops_identity(A, B):
    """Section 2.4: sum over k of nnz(A(:,k)) * nnz(B(k,:))."""
    ra, ca, _ = triples(A)
    rb, cb, _ = triples(B)
    return int(np.dot(np.bincount(ca, minlength=A.ncols).astype(np.int64),
                      np.bincount(rb, minlength=B.nrows).astype(np.int64)))


@pytest.mark.parametrize("semiring", SEMIRINGS)
def test_flops_identity_and_size_bound(semiring):
    for seed, (m, k, n, d) in enumerate([(50, 60, 40, 0.05), (200, 100, 300, 0.01), (7, 500, 9, 0.3)]):
        for fmt in ("csr", "dcsc"):
            A = W.random_sparse(m, k, d, semiring, fmt, seed)
            B = W.random_sparse(k, n, d, semiring, fmt, seed + 50)
            C, flops = oracle.spgemm(semiring, A, B)
            assert flops == _flops_identity(A, B)
            assert C.nnz <= flops
    A = W.rmat_matrix(10, 8, semiring, "csr", seed=1)
    C, flops = oracle.spgemm(semiring, A, A)
    assert flops == _flops_identity(A, A)
    assert C.nnz <= flops


@pytest.mark.parametrize("semiring", SEMIRINGS)
@pytest.mark.parametrize("fmt", ["csr", "dcsc"])
def test_identity_and_permutation_exact(semiring, fmt):
    n = 256
    A = W.rmat_matrix(8, 8, semiring, fmt, seed=7)
    I = W.identity_matrix(n, fmt, semiring)
    for L, R in ((A, I), (I, A)):
        C, flops = oracle.spgemm(semiring, L, R)
        assert flops == A.nnz
        assert_same(C, A, semiring, 0.0)
    Q = W.permutation_matrix(n, 3, fmt, semiring)
    q = W.permutation_matrix(n, 3, "csr", semiring).idx.astype(np.int64)  # Q(i, q[i]) stored
    r, c, v = triples(A)
    # (A Q)(r, q[l]) = A(r, l)
    AQ = W.from_triples(r, q[c], v, n, n, "csr", semiring)
    C, _ = oracle.spgemm(semiring, A, Q)
    assert_same(C, AQ, semiring, 0.0)
    # (Q A)(i, c) = A(q[i], c), so an entry (l, c) of A lands at row q^-1(l)
    qinv = np.empty(n, dtype=np.int64)
    qinv[q] = np.arange(n)
    QA = W.from_triples(qinv[r], c, v, n, n, "csr", semiring)
    C, _ = oracle.spgemm(semiring, Q, A)
    assert_same(C, QA, semiring, 0.0)


@pytest.mark.parametrize("n", [4, 6, 8, 12])
def test_galerkin_closed_form(n):
    """R (L_n P) = 4 L_{n/2} exactly for the 2x2x2 aggregation P and R = P^T."""
    L = W.laplacian_7pt(n, "csr")
    P = W.aggregation_p(n, "csr")
    R = W.transpose(P, "csr")
    AP, f1 = oracle.spgemm("plus_times_f64", L, P)
    RAP, f2 = oracle.spgemm("plus_times_f64", R, AP)
    assert f1 == L.nnz  # P has one entry per row
    assert f2 == AP.nnz  # R has one entry per column
    Lc = W.laplacian_7pt(n // 2, "csr")
    Lc.val = Lc.val * 4.0
    assert_same(RAP, Lc, "plus_times_f64", 0.0)


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32", "or_and_bool"])
def test_symmetric_permutation(semiring):
    """(P A P^T)(P A P^T) = P (A A) P^T (the relabelling of Section 7.1)."""
    n = 512
    A = W.rmat_matrix(9, 8, semiring, "csr", seed=9)
    perm = np.random.default_rng(4).permutation(n)
    r, c, v = triples(A)
    PA = W.from_triples(perm[r], perm[c], v, n, n, "csr", semiring)
    C, _ = oracle.spgemm(semiring, A, A)
    CP, _ = oracle.spgemm(semiring, PA, PA)
    r2, c2, v2 = triples(C)
    PC = W.from_triples(perm[r2], perm[c2], v2, n, n, "csr", semiring)
    assert_same(CP, PC, semiring, 1e-12)


def test_summa_block_identity():
    """Sum over stages of A_0k A_k0 equals block (0,0) of A'A' (Section 3.2)."""
    scale, grid = 10, 4
    a_blocks, b_blocks = W.summa_share(scale, 8, grid, (0, 0), seed=2)
    b = (1 << scale) // grid
    acc = {}
    total_flops = 0
    for k in range(grid):
        Ck, fk = oracle.spgemm("plus_times_f64", a_blocks[k], b_blocks[k])
        total_flops += fk
        r, c, v = triples(Ck)
        for q in range(r.size):
            key = (int(r[q]), int(c[q]))
            acc[key] = acc.get(key, 0.0) + float(v[q])
    keys = sorted(acc)
    merged = W.from_triples(np.array([x[0] for x in keys]), np.array([x[1] for x in keys]),
                            np.array([acc[x] for x in keys]), b, b, "csr")
    # strips: A(I-block, :) and A(:, J-block) as full-width operands
    ra, ca, va = [], [], []
    rb, cb, vb = [], [], []
    for k in range(grid):
        r, c, v = triples(a_blocks[k])
        ra.append(r); ca.append(c + k * b); va.append(v)
        r, c, v = triples(b_blocks[k])
        rb.append(r + k * b); cb.append(c); vb.append(v)
    SA = W.from_triples(np.concatenate(ra), np.concatenate(ca), np.concatenate(va), b, grid * b, "dcsc")
    SB = W.from_triples(np.concatenate(rb), np.concatenate(cb), np.concatenate(vb), grid * b, b, "dcsc")
    C, flops = oracle.spgemm("plus_times_f64", SA, SB)
    assert flops == total_flops
    assert_same(C, merged, "plus_times_f64", 1e-12)


@pytest.mark.parametrize("semiring", SEMIRINGS)
def test_edge_shapes(semiring):
    for fmt in ("csr", "csc", "dcsr", "dcsc"):
        # empty operands, zero inner dimension, 1 x 1, empty vectors
        E = W.from_triples([], [], W.random_values(np.random.default_rng(0), 0, semiring), 5, 0, fmt, semiring)
        F = W.from_triples([], [], W.random_values(np.random.default_rng(0), 0, semiring), 0, 3, fmt, semiring)
        C, flops = oracle.spgemm(semiring, E, F)
        assert flops == 0 and C.nnz == 0 and C.nrows == 5 and C.ncols == 3
        one = W.random_values(np.random.default_rng(1), 1, semiring)
        X = W.from_triples([0], [0], one, 1, 1, fmt, semiring)
        C, flops = oracle.spgemm(semiring, X, X)
        assert flops == 1 and C.nnz == 1
        A = W.random_sparse(30, 40, 0.0, semiring, fmt, 1)
        B = W.random_sparse(40, 20, 0.2, semiring, fmt, 2)
        C, flops = oracle.spgemm(semiring, A, B)
        assert flops == 0 and C.nnz == 0


@pytest.mark.parametrize("semiring", SEMIRINGS)
def test_formats_agree(semiring):
    A = W.rmat_matrix(8, 8, semiring, "csr", seed=11)
    ref, fref = oracle.spgemm(semiring, A, A)
    for fa, fb in FMT_PAIRS:
        if (fa in ("csr", "dcsr")) != (fb in ("csr", "dcsr")):
            continue
        C, f = oracle.spgemm(semiring, W.to_format(A, fa, semiring), W.to_format(A, fb, semiring))
        assert f == fref
        assert_canonical(C)
        # the column-major runs accumulate in a different order than the row-major one
        assert_same(C, ref, semiring, 1e-12, f"{fa},{fb}")


@pytest.mark.parametrize("semiring", ["plus_times_f64", "plus_times_f32", "min_plus_i32", "or_and_bool"])
@pytest.mark.parametrize("fmt", ["csr", "csc", "dcsr", "dcsc"])
def test_threaded_driver_equals_serial(semiring, fmt):
    """The threaded driver only distributes slices of the streamed vectors over
    host threads: its output is bit-identical to the single-threaded oracle's."""
    A = W.to_format(W.rmat_matrix(11, 8, semiring, "csr", seed=3), fmt, semiring)
    C1, f1 = oracle.spgemm(semiring, A, A)
    C2, f2 = oracle.spgemm_threads(semiring, A, A, threads=5, chunks_per_thread=3)
    assert f1 == f2 and C1.fmt == C2.fmt and C1.nnz == C2.nnz
    for k in ("ptr", "idx", "val", "vid"):
        a, b = getattr(C1, k), getattr(C2, k)
        assert (a is None and b is None) or np.array_equal(a, b), k


# ---------------------------------------------------------------------------
# format utilities (Sections 2.2-2.4): triples -> compressed with repeated
# positions combined in list order, and format / orientation changes
from oracle import convert as OC  # noqa: E402


def _brute_coo(semiring, rows, cols, vals, nrows, ncols):
    """Dense dictionary of positions, values combined in list order one by one."""
    acc = {}
    for i in range(len(rows)):
        key = (int(rows[i]), int(cols[i]))
        x = None if vals is None else vals[i]
        if key not in acc:
            acc[key] = x
        elif semiring == "min_plus_i32":
            acc[key] = min(acc[key], x)
        elif x is not None:
            acc[key] = acc[key] + x  # numpy scalar add in the value type
    return acc


@pytest.mark.parametrize("semiring", ["plus_times_f64", "plus_times_f32", "min_plus_i32", "or_and_bool"])
@pytest.mark.parametrize("fmt", ["csr", "csc", "dcsr", "dcsc"])
def test_coo_to_compressed_brute_force(semiring, fmt):
    rng = np.random.default_rng(11)
    nrows, ncols, n = 13, 9, 400  # about 3.4 occurrences per position: long runs
    rows = rng.integers(0, nrows, n)
    cols = rng.integers(0, ncols, n)
    vals = W.random_values(rng, n, semiring)
    M = OC.coo_to_compressed(semiring, rows, cols, vals, nrows, ncols, fmt)
    assert_canonical(M)
    acc = _brute_coo(semiring, rows, cols, vals, nrows, ncols)
    r, c, v = OC.triples(M)
    assert len(r) == len(acc)
    for k in range(len(r)):
        want = acc[(int(r[k]), int(c[k]))]
        if v is not None:
            assert v[k] == want and v.dtype == want.dtype, (k, v[k], want)


def test_coo_fold_order_is_left_to_right():
    # 1 + 2^-53 + 2^-53 + ... : a left fold loses every small term, a pairwise sum keeps some
    vals = np.array([1.0] + [2.0 ** -53] * 6)
    M = OC.coo_to_compressed("plus_times_f64", np.zeros(7, np.int64), np.zeros(7, np.int64), vals, 1, 1, "csr")
    assert M.val[0] == 1.0
    M = OC.coo_to_compressed("plus_times_f64", np.zeros(7, np.int64), np.zeros(7, np.int64), vals[::-1].copy(), 1, 1,
                             "csr")
    assert M.val[0] == 1.0 + 6 * 2.0 ** -53


def test_coo_to_compressed_matches_scipy_on_exact_values():
    rng = np.random.default_rng(2)
    rows = rng.integers(0, 300, 5000)
    cols = rng.integers(0, 200, 5000)
    vals = rng.integers(1, 9, 5000).astype(np.float64)  # small integers: every order sums exactly
    M = OC.coo_to_compressed("plus_times_f64", rows, cols, vals, 300, 200, "csr")
    S = sp.coo_matrix((vals, (rows, cols)), shape=(300, 200)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    assert np.array_equal(M.ptr, S.indptr) and np.array_equal(M.idx, S.indices) and np.array_equal(M.val, S.data)


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32", "or_and_bool"])
def test_convert_is_the_transpose_of_storage(semiring):
    A = W.rmat_matrix(10, 8, semiring, "csr", seed=9)
    S = sp.csr_matrix(((A.val if A.val is not None else np.ones(A.nnz)), A.idx, A.ptr), shape=(A.nrows, A.ncols))
    for fmt in ("csc", "dcsc", "dcsr", "csr"):
        B = OC.convert(semiring, A, fmt)
        assert_canonical(B)
        back = OC.convert(semiring, B, "csr")
        assert np.array_equal(back.ptr, A.ptr) and np.array_equal(back.idx, A.idx)
        if A.val is not None:
            assert np.array_equal(back.val, A.val)
    C = OC.convert(semiring, A, "csc")
    T = S.T.tocsr()  # CSR of A^T holds the arrays of CSC of A
    T.sort_indices()
    assert np.array_equal(C.ptr, T.indptr) and np.array_equal(C.idx, T.indices)


# ---------------------------------------------------------------------------
# masked multi-level BFS (Section 6.2.2)
from oracle import bfs as OB  # noqa: E402


def test_bfs_levels_match_scipy_depths():
    """Depth of every reached vertex equals scipy's BFS depth (from its
    predecessor tree) on the graph whose edge k -> i is A(i, k)."""
    from scipy.sparse import csgraph
    A = W.rmat_matrix(10, 4, "or_and_bool", "csc", seed=13)
    G = sp.csc_matrix((np.ones(A.nnz), A.idx, A.ptr), shape=(A.nrows, A.ncols))
    src = [0, 5, 77, 1023]
    lv = OB.bfs_levels(A, src)
    for c, s in enumerate(src):
        order, pred = csgraph.breadth_first_order(G.T.tocsr(), s, directed=True, return_predecessors=True)
        depth = {int(s): 0}
        for v in order[1:]:
            depth[int(v)] = depth[int(pred[v])] + 1
        mine = {int(v): d for d, L in enumerate(lv[c]) for v in L}
        assert mine == depth


def test_bfs_levels_on_a_path_and_a_cycle():
    # path 0 -> 1 -> 2 -> 3 (A(i, k) = 1 for i = k + 1), and the cycle closing it
    n = 4
    P = W.from_triples(np.arange(1, n), np.arange(0, n - 1), None, n, n, "csc", "or_and_bool")
    lv = OB.bfs_levels(P, [0, 2])
    assert [list(x) for x in lv[0]] == [[0], [1], [2], [3]]
    assert [list(x) for x in lv[1]] == [[2], [3]]
    C = W.from_triples(np.array([1, 2, 3, 0]), np.array([0, 1, 2, 3]), None, n, n, "csc", "or_and_bool")
    lv = OB.bfs_levels(C, [1])
    assert [list(x) for x in lv[0]] == [[1], [2], [3], [0]]  # the cycle back to 1 is masked out
    assert len(OB.bfs_levels(C, [1], max_levels=2)[0]) == 3
