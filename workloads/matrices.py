"""Neutral host-side sparse matrix container and canonicalisation from triples.

Formats (Section 2.2-2.3 of the paper; 0-based ids here, the paper is 1-based):

* ``csr`` / ``csc``: a dense array of sparse vectors. ``ptr`` has one entry per
  row (csr) or column (csc) plus one; ``idx`` holds the minor ids.
* ``dcsr`` / ``dcsc``: doubly compressed, a sparse array of sparse vectors.
  ``vid`` (the paper's JC for dcsc) lists the major ids of the non-empty
  vectors in ascending order, ``ptr`` (the paper's CP) has ``len(vid) + 1``
  entries, and ``idx``/``val`` are the paper's IR/NUM.

Every matrix built here is canonical: minor ids strictly increasing inside
each vector, ``vid`` strictly increasing, every doubly compressed vector
non-empty, and no stored value equal to the semiring's additive identity.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

# value dtype per semiring name; None = pattern only
VALUE_DTYPES = {
    "plus_times_f64": np.float64,
    "plus_times_f32": np.float32,
    "min_plus_i32": np.int32,
    "or_and_bool": None,
}

# how duplicate coordinates of a generated triple list are combined
_COMBINE = {
    "plus_times_f64": "sum",
    "plus_times_f32": "sum",
    "min_plus_i32": "min",
    "or_and_bool": "or",
}

ROW_MAJOR = ("csr", "dcsr")
COL_MAJOR = ("csc", "dcsc")
FORMATS = ROW_MAJOR + COL_MAJOR


@dataclass
class SpMat:
    fmt: str
    nrows: int
    ncols: int
    ptr: np.ndarray            # int64, nvec + 1
    idx: np.ndarray            # int32, nnz
    val: Optional[np.ndarray]  # nnz values, or None for a boolean pattern
    vid: Optional[np.ndarray] = None  # int32 major ids (doubly compressed only)

    @property
    def nnz(self) -> int:
        return int(self.idx.shape[0])

    @property
    def nvec(self) -> int:
        return int(self.ptr.shape[0] - 1)

    @property
    def row_major(self) -> bool:
        return self.fmt in ROW_MAJOR

    @property
    def doubly(self) -> bool:
        return self.fmt in ("dcsr", "dcsc")

    @property
    def major_dim(self) -> int:
        return self.nrows if self.row_major else self.ncols

    @property
    def minor_dim(self) -> int:
        return self.ncols if self.row_major else self.nrows

    def major_ids(self) -> np.ndarray:
        """Major id of every stored vector."""
        if self.doubly:
            return self.vid
        return np.arange(self.nvec, dtype=np.int32)

    def triples(self):
        """(rows, cols, vals) in storage order."""
        lens = np.diff(self.ptr)
        major = np.repeat(self.major_ids().astype(np.int64), lens)
        minor = self.idx.astype(np.int64)
        if self.row_major:
            return major, minor, self.val
        return minor, major, self.val


def random_values(rng: np.random.Generator, n: int, semiring: str):
    """Values of generated entries: f64/f32 uniform(0,1), int32 uniform[1,100]."""
    dt = VALUE_DTYPES[semiring]
    if dt is None:
        return None
    if dt == np.int32:
        return rng.integers(1, 101, size=n, dtype=np.int32)
    if dt == np.float32:
        v = rng.random(n, dtype=np.float32)
        # uniform(0,1) may return exactly 0; keep entries strictly positive
        return np.where(v == 0, np.float32(2.0 ** -24), v).astype(np.float32)
    v = rng.random(n)
    return np.where(v == 0, 2.0 ** -53, v)


def from_triples(rows, cols, vals, nrows: int, ncols: int, fmt: str,
                 semiring: str = "plus_times_f64") -> SpMat:
    """Canonical matrix from a triple list; duplicates combined in list order
    (a left fold: ((v1 + v2) + v3) + ...)."""
    if fmt not in FORMATS:
        raise ValueError(f"unknown format {fmt}")
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if rows.shape != cols.shape:
        raise ValueError("rows/cols length mismatch")
    if rows.size and (rows.min() < 0 or rows.max() >= nrows or cols.min() < 0 or cols.max() >= ncols):
        raise ValueError("triple out of range")
    row_major = fmt in ROW_MAJOR
    major, minor = (rows, cols) if row_major else (cols, rows)
    minor_dim = ncols if row_major else nrows
    major_dim = nrows if row_major else ncols
    key = major * np.int64(minor_dim) + minor
    order = np.argsort(key, kind="stable")
    key_s = key[order]
    if key_s.size:
        head = np.empty(key_s.size, dtype=bool)
        head[0] = True
        np.not_equal(key_s[1:], key_s[:-1], out=head[1:])
        starts = np.flatnonzero(head)
    else:
        starts = np.zeros(0, dtype=np.int64)
    ukey = key_s[starts]
    how = _COMBINE[semiring]
    dt = VALUE_DTYPES[semiring]
    if dt is None or vals is None:
        uval = None
    else:
        vs = np.asarray(vals, dtype=dt)[order]
        if how in ("sum", "min"):
            # left fold of each run of a repeated position, in list order
            op = np.add if how == "sum" else np.minimum
            uval = vs[starts].copy()
            lens = np.diff(np.append(starts, vs.size))
            live = np.flatnonzero(lens > 1)
            k = 1
            while live.size:
                uval[live] = op(uval[live], vs[starts[live] + k])
                k += 1
                live = live[lens[live] > k]
            uval = uval.astype(dt, copy=False)
        else:
            uval = None
    umaj = (ukey // minor_dim).astype(np.int64)
    umin = (ukey % minor_dim).astype(np.int32)
    if fmt in ("csr", "csc"):
        counts = np.bincount(umaj, minlength=major_dim).astype(np.int64)
        ptr = np.zeros(major_dim + 1, dtype=np.int64)
        np.cumsum(counts, out=ptr[1:])
        vid = None
    else:
        if umaj.size:
            vhead = np.empty(umaj.size, dtype=bool)
            vhead[0] = True
            np.not_equal(umaj[1:], umaj[:-1], out=vhead[1:])
            vstarts = np.flatnonzero(vhead)
        else:
            vstarts = np.zeros(0, dtype=np.int64)
        vid = umaj[vstarts].astype(np.int32)
        ptr = np.append(vstarts, umaj.size).astype(np.int64)
    return SpMat(fmt, int(nrows), int(ncols), ptr, umin, uval, vid)


def to_format(M: SpMat, fmt: str, semiring: str = "plus_times_f64") -> SpMat:
    """Re-encode a canonical matrix in another format (no duplicates exist)."""
    if fmt == M.fmt:
        return M
    r, c, v = M.triples()
    return from_triples(r, c, v, M.nrows, M.ncols, fmt, semiring)
