"""CPU oracle for C = A (x) B over a semiring (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never imports it and shares no code
with it; it is the independent reference the GPU results are compared with.

``spgemm(semiring, A, B)`` returns ``(C, flops)``. It follows the classical
Gustavson column-by-column algorithm with a dense sparse accumulator
(paper, Section 1 and Section 3.3); the C source states the details.
``flops`` counts one per nonzero multiplication (the paper's definition in
Section 1), which equals the sum over k of nnz(A(:,k)) * nnz(B(k,:))
(Section 2.4).

Operands are duck-typed: any object with ``fmt`` ("csr", "csc", "dcsr",
"dcsc"), ``nrows``, ``ncols``, ``ptr`` (int64), ``idx`` (int32), ``val``
(or None) and, for the doubly compressed formats, ``vid`` (int32 major ids).
Both operands must have the same orientation (row-major or column-major).
The result has the orientation of the operands; it is doubly compressed when
the streamed operand is (B for column-major, A for row-major), else plain
compressed with a full pointer array.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import types

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SEMIRINGS = {
    "plus_times_f64": (0, np.float64),
    "plus_times_f32": (1, np.float32),
    "min_plus_i32": (2, np.int32),
    "or_and_bool": (3, None),
}


class _Vecs(ctypes.Structure):
    _fields_ = [
        ("nvec", ctypes.c_int64),
        ("vid", ctypes.c_void_p),
        ("ptr", ctypes.c_void_p),
        ("idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("nvec", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("flops", ctypes.c_int64),
        ("vid", ctypes.c_void_p),
        ("ptr", ctypes.c_void_p),
        ("idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (plain -O2, single thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_colwise.restype = ctypes.c_int
        lib.orc_colwise.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                    ctypes.POINTER(_Vecs), ctypes.POINTER(_Vecs),
                                    ctypes.POINTER(_Result)]
        lib.orc_free.restype = None
        lib.orc_free.argtypes = [ctypes.POINTER(_Result)]
        _lib = lib
    return _lib


def _vecs(M, vdt, keep):
    ptr = np.ascontiguousarray(M.ptr, dtype=np.int64)
    idx = np.ascontiguousarray(M.idx, dtype=np.int32)
    keep += [ptr, idx]
    v = _Vecs()
    v.nvec = ptr.shape[0] - 1
    v.ptr = ptr.ctypes.data
    v.idx = idx.ctypes.data if idx.size else None
    if M.fmt in ("dcsr", "dcsc"):
        vid = np.ascontiguousarray(M.vid, dtype=np.int32)
        keep.append(vid)
        v.vid = vid.ctypes.data if vid.size else None
        if not vid.size:
            v.vid = None
            v.nvec = 0
    else:
        v.vid = None
    if vdt is not None:
        val = np.ascontiguousarray(M.val, dtype=vdt)
        keep.append(val)
        v.val = val.ctypes.data if val.size else None
    else:
        v.val = None
    return v


def spgemm(semiring: str, A, B):
    """Return (C, flops) for C = A (x) B; see the module docstring."""
    return _spgemm(semiring, A, B, None)


def spgemm_threads(semiring: str, A, B, threads: int = None, chunks_per_thread: int = 8):
    """The same (C, flops) as ``spgemm``, computed on several host threads.

    The streamed vectors (columns of B, or rows of A row-major) are cut into
    consecutive slices; every slice runs the same single-threaded C routine
    (its own accumulator, every output vector summed in ascending k exactly as
    in ``spgemm``) on a thread of a pool (ctypes releases the interpreter lock
    during the call), and the slices' outputs are concatenated in order. Only
    the work is distributed; no output value is computed differently.
    """
    import concurrent.futures as cf
    if threads is None:
        threads = os.cpu_count() or 1
    col = A.fmt in ("csc", "dcsc")
    S = B if col else A
    nvec = int(np.asarray(S.ptr).shape[0] - 1)
    if S.fmt in ("dcsr", "dcsc") and (S.vid is None or len(S.vid) == 0):
        nvec = 0
    if threads <= 1 or nvec < 2:
        return _spgemm(semiring, A, B, None)
    # slices of about equal stored entries
    ptr = np.asarray(S.ptr, dtype=np.int64)
    nslices = max(1, min(nvec, threads * chunks_per_thread))
    cuts = np.searchsorted(ptr, np.linspace(0, ptr[-1], nslices + 1)[1:-1]).tolist()
    bounds = sorted(set([0] + [min(max(int(c), 0), nvec) for c in cuts] + [nvec]))
    slices = list(zip(bounds[:-1], bounds[1:]))
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda ab: _spgemm(semiring, A, B, ab, raw=True), slices))
    return _assemble(semiring, A, B, parts)


def _spgemm(semiring, A, B, rng, raw=False):
    code, vdt = SEMIRINGS[semiring]
    col = A.fmt in ("csc", "dcsc")
    if col != (B.fmt in ("csc", "dcsc")):
        raise ValueError("operands must share an orientation")
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    keep = []
    if col:
        G, S, gfirst, m, major_dim = A, B, 1, A.nrows, B.ncols
    else:
        G, S, gfirst, m, major_dim = B, A, 0, B.ncols, A.nrows
    gv = _vecs(G, vdt, keep)
    sv = _vecs(S, vdt, keep)
    t0 = 0
    if rng is not None:
        # slice [t0, t1) of the streamed vectors: pointer and id arrays start at
        # t0; the entry offsets in ptr stay absolute, so idx/val are unchanged
        t0, t1 = rng
        sv.nvec = t1 - t0
        sv.ptr = (sv.ptr or 0) + 8 * t0
        if sv.vid:
            sv.vid = sv.vid + 4 * t0
    res = _Result()
    lib = _load()
    rc = lib.orc_colwise(code, gfirst, int(m), ctypes.byref(gv), ctypes.byref(sv), ctypes.byref(res))
    if rc != 0:
        lib.orc_free(ctypes.byref(res))
        raise RuntimeError(f"oracle failed with code {rc}")
    try:
        nv, nnz = res.nvec, res.nnz
        vid = np.ctypeslib.as_array(ctypes.cast(res.vid, ctypes.POINTER(ctypes.c_int32)), (max(nv, 1),))[:nv].copy()
        vptr = np.ctypeslib.as_array(ctypes.cast(res.ptr, ctypes.POINTER(ctypes.c_int64)), (nv + 1,)).copy()
        if nnz:
            idx = np.ctypeslib.as_array(ctypes.cast(res.idx, ctypes.POINTER(ctypes.c_int32)), (nnz,)).copy()
        else:
            idx = np.zeros(0, dtype=np.int32)
        if vdt is None:
            val = None
        elif nnz:
            ctype = {np.float64: ctypes.c_double, np.float32: ctypes.c_float, np.int32: ctypes.c_int32}[vdt]
            val = np.ctypeslib.as_array(ctypes.cast(res.val, ctypes.POINTER(ctype)), (nnz,)).copy()
        else:
            val = np.zeros(0, dtype=vdt)
        flops = int(res.flops)
    finally:
        lib.orc_free(ctypes.byref(res))
    if S.fmt not in ("dcsr", "dcsc"):
        vid = vid + np.int32(t0)  # a slice numbers its plain vectors from 0
    if raw:
        return vid, vptr, idx, val, flops
    return _finish(A, B, S, col, major_dim, vid, vptr, idx, val, nnz, flops)


def _assemble(semiring, A, B, parts):
    col = A.fmt in ("csc", "dcsc")
    S = B if col else A
    major_dim = B.ncols if col else A.nrows
    vids, ptrs, idxs, vals = [], [], [], []
    off = 0
    flops = 0
    for vid, vptr, idx, val, f in parts:
        vids.append(vid)
        ptrs.append(vptr[1:] + off)
        idxs.append(idx)
        vals.append(val)
        off += int(vptr[-1])
        flops += f
    vid = np.concatenate(vids).astype(np.int32)
    vptr = np.concatenate([np.zeros(1, np.int64)] + ptrs)
    idx = np.concatenate(idxs).astype(np.int32)
    val = None if vals[0] is None else np.concatenate(vals)
    return _finish(A, B, S, col, major_dim, vid, vptr, idx, val, off, flops)


def _finish(A, B, S, col, major_dim, vid, vptr, idx, val, nnz, flops):
    nv = vid.shape[0]
    doubly = S.fmt in ("dcsr", "dcsc")
    if col:
        fmt = "dcsc" if doubly else "csc"
    else:
        fmt = "dcsr" if doubly else "csr"
    if doubly:
        ptr = vptr
        out_vid = vid
    else:
        counts = np.zeros(major_dim, dtype=np.int64)
        counts[vid] = np.diff(vptr)
        ptr = np.zeros(major_dim + 1, dtype=np.int64)
        np.cumsum(counts, out=ptr[1:])
        out_vid = None
    nrows = A.nrows
    ncols = B.ncols
    C = types.SimpleNamespace(fmt=fmt, nrows=nrows, ncols=ncols, ptr=ptr, idx=idx, val=val,
                              vid=out_vid, nnz=int(nnz), nvec=int(ptr.shape[0] - 1))
    return C, flops
