"""Seeded generators for the synthetic workloads (R-MAT, 3D grid, SUMMA share, BFS)."""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .matrices import SpMat, VALUE_DTYPES, from_triples, random_values

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)

# multiplicative identity of each semiring's value type (entries of identity
# and permutation matrices); None = boolean pattern
_ONE = {
    "plus_times_f64": 1.0,
    "plus_times_f32": 1.0,
    "min_plus_i32": 0,
    "or_and_bool": None,
}


def _torch():
    import torch  # local import: generators are usable without a GPU
    return torch


def rmat_edges(scale: int, edge_factor: int, abcd: Sequence[float] = RMAT_ABCD,
               seed: int = 1, device: str = "cpu", batch: int = 1 << 24):
    """R-MAT edge list (Section 5.1.1): ``edge_factor * 2**scale`` directed edges.

    For every edge and every one of the ``scale`` levels, one uniform draw
    picks a quadrant of the 2x2 generator: a -> (0,0), b -> (0,1),
    c -> (1,0), d -> (1,1); the chosen row/column bit is set at that level,
    most significant bit first. Self loops and repeated edges are kept.
    Returns torch int64 tensors (rows, cols) on ``device``.
    """
    torch = _torch()
    a, b, c, d = (float(x) for x in abcd)
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("R-MAT probabilities must sum to 1")
    m = int(edge_factor) << int(scale)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    rows = torch.empty(m, dtype=torch.int64, device=device)
    cols = torch.empty(m, dtype=torch.int64, device=device)
    t1, t2, t3 = a, a + b, a + b + c
    for s in range(0, m, batch):
        nb = min(batch, m - s)
        r = torch.zeros(nb, dtype=torch.int64, device=device)
        q = torch.zeros(nb, dtype=torch.int64, device=device)
        for level in range(scale):
            u = torch.rand(nb, generator=g, device=device, dtype=torch.float64)
            bit = 1 << (scale - 1 - level)
            rbit = u >= t2
            cbit = ((u >= t1) & (u < t2)) | (u >= t3)
            r |= rbit.to(torch.int64) * bit
            q |= cbit.to(torch.int64) * bit
        rows[s:s + nb] = r
        cols[s:s + nb] = q
    return rows, cols


def _edge_values_torch(m: int, semiring: str, seed: int, device: str):
    """Per-edge values in generation order, drawn on ``device``."""
    torch = _torch()
    dt = VALUE_DTYPES[semiring]
    if dt is None:
        return None
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 7919 + 17)
    if dt == np.int32:
        return torch.randint(1, 101, (m,), generator=g, device=device, dtype=torch.int32)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    v = torch.rand(m, generator=g, device=device, dtype=tdt)
    tiny = 2.0 ** -24 if dt == np.float32 else 2.0 ** -53
    return torch.where(v == 0, torch.full_like(v, tiny), v)


def rmat_matrix(scale: int, edge_factor: int, semiring: str = "plus_times_f64",
                fmt: str = "csr", seed: int = 1, abcd: Sequence[float] = RMAT_ABCD,
                device: str = "cpu") -> SpMat:
    """Square R-MAT matrix n = 2**scale, duplicates combined by the semiring's add."""
    rows, cols = rmat_edges(scale, edge_factor, abcd, seed, device)
    vals = _edge_values_torch(rows.numel(), semiring, seed, device)
    n = 1 << scale
    r = rows.cpu().numpy()
    c = cols.cpu().numpy()
    v = None if vals is None else vals.cpu().numpy()
    return from_triples(r, c, v, n, n, fmt, semiring)


def laplacian_7pt(n: int, fmt: str = "csr", semiring: str = "plus_times_f64") -> SpMat:
    """7-point finite-difference Laplacian on an n x n x n grid (Section 5.1.3).

    Lexicographic numbering id = x + n*(y + n*z); diagonal 6, -1 for each of
    the six face neighbours that lie inside the grid (Dirichlet truncation).
    """
    N = n ** 3
    ids = np.arange(N, dtype=np.int64)
    x = ids % n
    y = (ids // n) % n
    z = ids // (n * n)
    rows = [ids]
    cols = [ids]
    vals = [np.full(N, 6.0)]
    for dim, coord, stride in ((0, x, 1), (1, y, n), (2, z, n * n)):
        for step in (-1, 1):
            ok = (coord + step >= 0) & (coord + step < n)
            src = ids[ok]
            rows.append(src)
            cols.append(src + step * stride)
            vals.append(np.full(src.size, -1.0))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    if VALUE_DTYPES[semiring] is None:
        v = None
    elif VALUE_DTYPES[semiring] != np.float64:
        v = v.astype(VALUE_DTYPES[semiring])
    return from_triples(r, c, v, N, N, fmt, semiring)


def aggregation_p(n: int, fmt: str = "csr", semiring: str = "plus_times_f64") -> SpMat:
    """2x2x2 aggregation prolongation P (N x N/8, entries one).

    Fine point (z, y, x) belongs to the aggregate (z//2, y//2, x//2), numbered
    lexicographically on the (n/2)^3 coarse grid.
    """
    if n % 2:
        raise ValueError("grid size must be even")
    N = n ** 3
    h = n // 2
    ids = np.arange(N, dtype=np.int64)
    x = ids % n
    y = (ids // n) % n
    z = ids // (n * n)
    agg = (x // 2) + h * ((y // 2) + h * (z // 2))
    one = _ONE[semiring]
    v = None if one is None else np.full(N, one, dtype=VALUE_DTYPES[semiring])
    return from_triples(ids, agg, v, N, h ** 3, fmt, semiring)


def transpose(M: SpMat, fmt: Optional[str] = None, semiring: str = "plus_times_f64") -> SpMat:
    """Explicit transpose (input preparation, e.g. R = P^T)."""
    r, c, v = M.triples()
    return from_triples(c, r, v, M.ncols, M.nrows, fmt or M.fmt, semiring)


def summa_share(scale: int, edge_factor: int, grid: int, proc: Tuple[int, int] = (0, 0),
                semiring: str = "plus_times_f64", seed: int = 24,
                abcd: Sequence[float] = RMAT_ABCD, device: str = "cpu",
                fmt: str = "dcsc") -> Tuple[List[SpMat], List[SpMat]]:
    """Operands of one Sparse SUMMA process (Sections 3.2, 3.5; relabelling Section 7.1).

    The R-MAT matrix A (n = 2**scale) is relabelled by a seeded random
    symmetric permutation (entry (u, v) moves to (pi(u), pi(v))), then cut
    into a ``grid`` x ``grid`` array of (n/grid)^2 blocks. Process (I, J)
    multiplies, at stage k, A_Ik by A_kJ. Returns the two lists
    ``[A_I0 .. A_I,grid-1]`` and ``[A_0J .. A_grid-1,J]`` with block-local ids.
    """
    torch = _torch()
    n = 1 << scale
    if n % grid:
        raise ValueError("grid must divide n")
    b = n // grid
    I, J = proc
    rows, cols = rmat_edges(scale, edge_factor, abcd, seed, device)
    vals = _edge_values_torch(rows.numel(), semiring, seed, device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 104729 + 3)
    perm = torch.randperm(n, generator=g, device=device)
    pu = perm[rows]
    pv = perm[cols]
    del rows, cols
    mask_a = (pu // b) == I
    mask_b = (pv // b) == J

    def blocks(mask, row_local: bool):
        r = pu[mask].cpu().numpy()
        c = pv[mask].cpu().numpy()
        v = None if vals is None else vals[mask].cpu().numpy()
        if row_local:
            r = r - I * b
            blk = c // b
            c = c - blk * b
        else:
            c = c - J * b
            blk = r // b
            r = r - blk * b
        order = np.argsort(blk, kind="stable")
        blk_s = blk[order]
        bounds = np.searchsorted(blk_s, np.arange(grid + 1))
        out = []
        for k in range(grid):
            sel = order[bounds[k]:bounds[k + 1]]
            out.append(from_triples(r[sel], c[sel], None if v is None else v[sel], b, b, fmt, semiring))
        return out

    a_blocks = blocks(mask_a, True)
    b_blocks = blocks(mask_b, False)
    return a_blocks, b_blocks


def bfs_frontier(n: int, k: int, seed: int = 5, A: Optional[SpMat] = None,
                 depth: int = 0, fmt: str = "csc") -> SpMat:
    """Boolean n x k frontier with one uniformly random source per column.

    depth 0: X(:, s) holds only the source. depth 1: X(:, s) is the pattern
    of column ``src_s`` of the column-major matrix A (the source's
    neighbours), a heavier frontier as in the deeper BFS levels of Section 6.2.2.
    """
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=k, dtype=np.int64)
    if depth == 0:
        return from_triples(src, np.arange(k, dtype=np.int64), None, n, k, fmt, "or_and_bool")
    if A is None or A.row_major or A.doubly:
        raise ValueError("depth-1 frontier needs a csc matrix A")
    rows, cols = [], []
    for s, u in enumerate(src):
        seg = A.idx[A.ptr[u]:A.ptr[u + 1]].astype(np.int64)
        if seg.size == 0:
            seg = np.array([u], dtype=np.int64)
        rows.append(seg)
        cols.append(np.full(seg.size, s, dtype=np.int64))
    return from_triples(np.concatenate(rows), np.concatenate(cols), None, n, k, fmt, "or_and_bool")


def poisson_arrivals(qps: float, count: int, seed: int = 11) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: exponential gaps of mean 1/qps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


def random_sparse(m: int, n: int, density: float, semiring: str = "plus_times_f64",
                  fmt: str = "csr", seed: int = 0) -> SpMat:
    """Erdos-Renyi style matrix (Section 5.1.2): each entry present with prob. density."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    r, c = np.nonzero(mask)
    v = random_values(rng, r.size, semiring)
    return from_triples(r, c, v, m, n, fmt, semiring)


def permutation_matrix(n: int, seed: Optional[int] = 0, fmt: str = "csr",
                       semiring: str = "plus_times_f64") -> SpMat:
    """Q with Q(i, q_i) = multiplicative identity; seed None gives the identity."""
    rows = np.arange(n, dtype=np.int64)
    if seed is None:
        cols = rows.copy()
    else:
        cols = np.random.default_rng(seed).permutation(n).astype(np.int64)
    one = _ONE[semiring]
    v = None if one is None else np.full(n, one, dtype=VALUE_DTYPES[semiring])
    return from_triples(rows, cols, v, n, n, fmt, semiring)


def identity_matrix(n: int, fmt: str = "csr", semiring: str = "plus_times_f64") -> SpMat:
    return permutation_matrix(n, None, fmt, semiring)
