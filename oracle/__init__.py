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
