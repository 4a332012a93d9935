"""CPU oracle of the format utilities (test infrastructure only; the same
import rules as the rest of ``oracle``).

``coo_to_compressed``: the compressed matrix of a triple list. The paper's
formats (Section 2.2: CSR/CSC; Section 2.3: DCSC, whose JC lists only the
non-empty columns) store each position once; positions that occur several
times in the list are combined with the semiring's add, in list order, as a
left fold ((v1 + v2) + v3) + ... Ids end ascending inside each vector.

``convert``: the same matrix in another of the four formats. Between the
two orientations this is the transpose of the storage (CSC of M holds the
arrays of CSR of M^T), the preprocessing step that makes a row-major product
column-wise (Section 2.4).

Plain numpy: a stable argsort (library primitive) orders the triples by
(major, minor); the fold walks each run of equal positions one step at a
time, in list order.
"""
from __future__ import annotations

import types

import numpy as np

VALUE_DTYPES = {"plus_times_f64": np.float64, "plus_times_f32": np.float32,
                "min_plus_i32": np.int32, "or_and_bool": None}
ROW_MAJOR = ("csr", "dcsr")


def _fold(semiring, v_sorted, starts, lens):
    """Left fold of every run [starts[r], starts[r] + lens[r]) of v_sorted, in order:
    step k adds the (k+1)-th value of every run longer than k."""
    res = v_sorted[starts].copy()
    op = np.minimum if semiring == "min_plus_i32" else np.add
    live = np.flatnonzero(lens > 1)
    k = 1
    while live.size:
        res[live] = op(res[live], v_sorted[starts[live] + k])
        k += 1
        live = live[lens[live] > k]
    return res


def coo_to_compressed(semiring, rows, cols, vals, nrows, ncols, fmt):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= nrows or cols.min() < 0 or cols.max() >= ncols):
        raise ValueError("triple out of range")
    rm = fmt in ROW_MAJOR
    major, minor = (rows, cols) if rm else (cols, rows)
    major_dim, minor_dim = (nrows, ncols) if rm else (ncols, nrows)
    key = major * np.int64(minor_dim) + minor
    order = np.argsort(key, kind="stable")
    ks = key[order]
    head = np.ones(ks.size, dtype=bool)
    if ks.size:
        head[1:] = ks[1:] != ks[:-1]
    starts = np.flatnonzero(head)
    lens = np.diff(np.append(starts, ks.size))
    ukey = ks[starts]
    dt = VALUE_DTYPES[semiring]
    uval = None
    if dt is not None:
        uval = _fold(semiring, np.asarray(vals, dtype=dt)[order], starts, lens).astype(dt)
    umaj = ukey // minor_dim
    umin = (ukey % minor_dim).astype(np.int32)
    if fmt in ("csr", "csc"):
        counts = np.bincount(umaj, minlength=major_dim).astype(np.int64)
        ptr = np.zeros(major_dim + 1, dtype=np.int64)
        np.cumsum(counts, out=ptr[1:])
        vid = None
    else:
        vh = np.ones(umaj.size, dtype=bool)
        if umaj.size:
            vh[1:] = umaj[1:] != umaj[:-1]
        vs = np.flatnonzero(vh)
        vid = umaj[vs].astype(np.int32)
        ptr = np.append(vs, umaj.size).astype(np.int64)
    return types.SimpleNamespace(fmt=fmt, nrows=int(nrows), ncols=int(ncols), ptr=ptr, idx=umin, val=uval, vid=vid)


def triples(M):
    """(rows, cols, vals) of a compressed matrix in storage order."""
    ptr = np.asarray(M.ptr, dtype=np.int64)
    lens = np.diff(ptr)
    if M.fmt in ("dcsr", "dcsc"):
        majors = np.asarray(M.vid, dtype=np.int64)
    else:
        majors = np.arange(lens.size, dtype=np.int64)
    maj = np.repeat(majors, lens)
    mnr = np.asarray(M.idx, dtype=np.int64)[ptr[0]:ptr[-1]]
    v = None if M.val is None else np.asarray(M.val)[ptr[0]:ptr[-1]]
    return (maj, mnr, v) if M.fmt in ROW_MAJOR else (mnr, maj, v)


def convert(semiring, M, fmt):
    """M (canonical, no repeated positions) in format `fmt`."""
    r, c, v = triples(M)
    return coo_to_compressed(semiring, r, c, v, M.nrows, M.ncols, fmt)
