"""Shared test utilities: triple extraction, canonical-form checks, comparisons."""
import numpy as np

INT32_MAX = np.iinfo(np.int32).max


def major_ids(M):
    if M.fmt in ("dcsr", "dcsc"):
        return np.asarray(M.vid, dtype=np.int64)
    return np.arange(len(M.ptr) - 1, dtype=np.int64)


def triples(M):
    """(rows, cols, vals) sorted by (row, col)."""
    ptr = np.asarray(M.ptr, dtype=np.int64)
    lens = np.diff(ptr)
    maj = np.repeat(major_ids(M), lens)
    mnr = np.asarray(M.idx, dtype=np.int64)[: ptr[-1]]
    if M.fmt in ("csr", "dcsr"):
        r, c = maj, mnr
    else:
        r, c = mnr, maj
    order = np.lexsort((c, r))
    v = None if M.val is None else np.asarray(M.val)[: ptr[-1]][order]
    return r[order], c[order], v


def assert_canonical(M):
    ptr = np.asarray(M.ptr, dtype=np.int64)
    assert ptr[0] == 0
    assert np.all(np.diff(ptr) >= 0)
    idx = np.asarray(M.idx, dtype=np.int64)[: ptr[-1]]
    lens = np.diff(ptr)
    seg = np.repeat(np.arange(len(lens)), lens)
    if idx.size > 1:
        same = seg[1:] == seg[:-1]
        assert np.all(idx[1:][same] > idx[:-1][same]), "minor ids not strictly increasing"
    minor_dim = M.ncols if M.fmt in ("csr", "dcsr") else M.nrows
    if idx.size:
        assert idx.min() >= 0 and idx.max() < minor_dim
    if M.fmt in ("dcsr", "dcsc"):
        vid = np.asarray(M.vid, dtype=np.int64)
        assert np.all(np.diff(vid) > 0)
        assert np.all(lens > 0), "doubly compressed vector is empty"


def assert_same(C, R, semiring, rtol=0.0, what=""):
    """Pattern equal and values equal (exact, or within rtol per entry)."""
    r1, c1, v1 = triples(C)
    r2, c2, v2 = triples(R)
    assert r1.shape == r2.shape, f"{what}: nnz {r1.size} vs {r2.size}"
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2), f"{what}: pattern differs"
    if semiring == "or_and_bool":
        return
    assert v1 is not None and v2 is not None
    if rtol == 0.0 or semiring == "min_plus_i32":
        assert np.array_equal(v1, v2), f"{what}: values differ"
    else:
        v1 = v1.astype(np.float64)
        v2 = v2.astype(np.float64)
        err = np.abs(v1 - v2)
        bad = err > rtol * np.abs(v2)
        assert not bad.any(), f"{what}: {bad.sum()} values beyond rtol {rtol}, worst {np.max(err / np.maximum(np.abs(v2), 1e-300))}"
