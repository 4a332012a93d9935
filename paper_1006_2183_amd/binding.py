"""ctypes binding of the C ABI in include/sg_spgemm.h (argument marshalling only).

PyTorch supplies device memory and the stream; every step of the product
runs in the library's HIP kernels. There is no CPU fallback: if the shared
library is missing, loading fails with an error that says how to build it.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgspgemm.so")
# the same library built with SG_CHECK=1 (invariant counters, see sg_plan_check)
CHECK_LIB_PATH = os.path.join(HERE, "libsgspgemm_check.so")

SEMIRINGS = {"plus_times_f64": 0, "plus_times_f32": 1, "min_plus_i32": 2, "or_and_bool": 3}
FORMATS = {"csr": 0, "csc": 1, "dcsr": 2, "dcsc": 3}
FORMAT_NAMES = {v: k for k, v in FORMATS.items()}
STATUS = {0: "SG_OK", -1: "SG_ERR_INVALID_ARG", -2: "SG_ERR_DIM_MISMATCH", -3: "SG_ERR_NOT_CANONICAL",
          -4: "SG_ERR_UNSUPPORTED", -5: "SG_ERR_WORKSPACE", -6: "SG_ERR_CAPACITY", -7: "SG_ERR_HIP",
          -8: "SG_ERR_OOM"}

EXPORTS = ["sg_tuning_default", "sg_status_string", "sg_last_error", "sg_spgemm_workspace_size", "sg_spgemm_symbolic",
           "sg_spgemm_numeric", "sg_spgemm_batched", "sg_plan_profile", "sg_plan_kernel_times", "sg_plan_destroy",
           "sg_validate", "sg_build_aux", "sg_plan_check", "sg_build_checked", "sg_coo_workspace_size",
           "sg_coo_compress", "sg_coo_emit", "sg_convert_workspace_size", "sg_convert", "sg_spgemm_symbolic_masked",
           "sg_mask_set", "sg_chain_workspace_size", "sg_chain_symbolic", "sg_convert_static",
           "sg_convert_static_bytes", "sg_autotune"]


class SgError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        msg = f"{where}: {STATUS.get(status, status)}"
        if detail:
            msg += f" [{detail}]"
        super().__init__(msg)
        self.status = status


class sg_semiring(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32)]


class sg_mat(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64),
                ("nvec", ctypes.c_int64), ("nnz", ctypes.c_int64), ("ptr", ctypes.c_void_p),
                ("vid", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class sg_mat_out(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64),
                ("cap_nnz", ctypes.c_int64), ("cap_vec", ctypes.c_int64), ("ptr", ctypes.c_void_p),
                ("vid", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class sg_mask(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("stride_words", ctypes.c_int64), ("complement", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class sg_tuning(ctypes.Structure):
    _fields_ = [("tiny_max_flops", ctypes.c_int32), ("mid_max_ub", ctypes.c_int32), ("mid_kind", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("block_threads", ctypes.c_int32), ("chunk_width", ctypes.c_int32),
                ("heavy_kind", ctypes.c_int32), ("force_tier", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("xcd_ranges", ctypes.c_int32),
                ("bitmap_mb", ctypes.c_int32),
                ("heavy_threads", ctypes.c_int32),
                ("heavy_lds_bytes", ctypes.c_int32),
                ("entry_mb", ctypes.c_int32),
                ("small_max_flops", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class sg_sym_info(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("flops", "nnz_ub", "nnz", "nvec", "max_vec_flops", "n_out_vec",
                                              "n_tiny", "n_mid", "n_heavy", "n_heavy_items")] + [
        ("tier_flops", ctypes.c_int64 * 3), ("tier_sent", ctypes.c_int64 * 3), ("tier_nnz", ctypes.c_int64 * 3),
        ("n_small", ctypes.c_int64)]

    def as_dict(self):
        d = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            d[f] = [int(x) for x in v] if f.startswith("tier_") else int(v)
        return d


_lib = None
_libs = {}


def load_library(path: Optional[str] = None):
    """Load the HIP library (no compute). Raises if it has not been built.

    The first call fixes the library the binding uses (the normal build unless
    ``use_library`` chose another); later calls return it."""
    global _lib
    if path is None:
        if _lib is not None:
            return _lib
        path = LIB_PATH
    if path in _libs:
        if _lib is None:
            _lib = _libs[path]
        return _libs[path]
    # torch ships its own HIP runtime under the same soname as the system one;
    # whichever is loaded first serves the whole process, so load torch's first
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing; build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.sg_tuning_default.restype = None
    lib.sg_tuning_default.argtypes = [ctypes.c_int32, P(sg_tuning)]
    lib.sg_status_string.restype = ctypes.c_char_p
    lib.sg_status_string.argtypes = [ctypes.c_int32]
    lib.sg_last_error.restype = ctypes.c_char_p
    lib.sg_last_error.argtypes = []
    lib.sg_spgemm_workspace_size.restype = ctypes.c_int
    lib.sg_spgemm_workspace_size.argtypes = [P(sg_semiring), ctypes.c_int32, P(sg_mat), P(sg_mat), ctypes.c_void_p,
                                             ctypes.c_int32, ctypes.c_int32, P(sg_tuning), P(ctypes.c_size_t)]
    lib.sg_spgemm_symbolic.restype = ctypes.c_int
    lib.sg_spgemm_symbolic.argtypes = [P(sg_semiring), ctypes.c_int32, P(sg_mat), P(sg_mat), ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.c_int32, P(sg_tuning), ctypes.c_void_p, ctypes.c_size_t,
                                       P(ctypes.c_void_p), P(sg_sym_info), ctypes.c_void_p]
    lib.sg_spgemm_numeric.restype = ctypes.c_int
    lib.sg_spgemm_numeric.argtypes = [ctypes.c_void_p, P(sg_mat_out), ctypes.c_void_p]
    lib.sg_spgemm_batched.restype = ctypes.c_int
    lib.sg_spgemm_batched.argtypes = [ctypes.c_void_p, P(sg_mat_out), ctypes.c_void_p]
    lib.sg_plan_profile.restype = ctypes.c_int
    lib.sg_plan_profile.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.sg_plan_kernel_times.restype = ctypes.c_int
    lib.sg_plan_kernel_times.argtypes = [ctypes.c_void_p, P(ctypes.c_double), ctypes.c_int32]
    lib.sg_plan_destroy.restype = ctypes.c_int
    lib.sg_plan_destroy.argtypes = [ctypes.c_void_p]
    lib.sg_validate.restype = ctypes.c_int
    lib.sg_validate.argtypes = [P(sg_mat), ctypes.c_void_p, ctypes.c_void_p]
    lib.sg_build_aux.restype = ctypes.c_int
    lib.sg_build_aux.argtypes = [P(sg_mat), ctypes.c_void_p, P(ctypes.c_int64), ctypes.c_void_p]
    lib.sg_plan_check.restype = ctypes.c_int
    lib.sg_plan_check.argtypes = [ctypes.c_void_p, P(ctypes.c_int64), ctypes.c_int32]
    lib.sg_build_checked.restype = ctypes.c_int32
    lib.sg_build_checked.argtypes = []
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.sg_coo_workspace_size.restype = ctypes.c_int
    lib.sg_coo_workspace_size.argtypes = [P(sg_semiring), i64, i64, i64, ctypes.c_int32, P(ctypes.c_size_t)]
    lib.sg_coo_compress.restype = ctypes.c_int
    lib.sg_coo_compress.argtypes = [P(sg_semiring), i64, i64, i64, vp, vp, vp, ctypes.c_int32, vp, ctypes.c_size_t,
                                    P(i64), P(i64), vp]
    lib.sg_coo_emit.restype = ctypes.c_int
    lib.sg_coo_emit.argtypes = [P(sg_semiring), i64, i64, i64, ctypes.c_int32, vp, ctypes.c_size_t, i64, i64,
                                P(sg_mat_out), vp]
    lib.sg_convert_workspace_size.restype = ctypes.c_int
    lib.sg_convert_workspace_size.argtypes = [P(sg_semiring), P(sg_mat), ctypes.c_int32, P(ctypes.c_size_t)]
    lib.sg_spgemm_symbolic_masked.restype = ctypes.c_int
    lib.sg_spgemm_symbolic_masked.argtypes = [P(sg_semiring), ctypes.c_int32, P(sg_mat), P(sg_mat), ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_int32, P(sg_mask), P(sg_tuning), ctypes.c_void_p,
                                              ctypes.c_size_t, P(ctypes.c_void_p), P(sg_sym_info), ctypes.c_void_p]
    lib.sg_chain_workspace_size.restype = ctypes.c_int
    lib.sg_chain_workspace_size.argtypes = [P(sg_semiring), ctypes.c_int32, P(sg_mat), P(sg_mat), P(sg_mat), ctypes.c_int32,
                                            P(sg_tuning), P(ctypes.c_size_t)]
    lib.sg_chain_symbolic.restype = ctypes.c_int
    lib.sg_chain_symbolic.argtypes = [P(sg_semiring), ctypes.c_int32, P(sg_mat), P(sg_mat), P(sg_mat), ctypes.c_int32,
                                      P(sg_tuning), ctypes.c_void_p, ctypes.c_size_t, P(ctypes.c_void_p), P(sg_sym_info),
                                      ctypes.c_void_p]
    lib.sg_convert_static.restype = ctypes.c_int
    lib.sg_convert_static.argtypes = [P(sg_semiring), P(sg_mat), ctypes.c_int32, P(sg_mat_out), P(i64), vp]
    lib.sg_autotune.restype = ctypes.c_int
    lib.sg_autotune.argtypes = [P(sg_semiring), ctypes.c_int32, P(sg_mat), P(sg_mat), vp, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P(sg_tuning), P(ctypes.c_double),
                                P(ctypes.c_double), vp]
    lib.sg_convert_static_bytes.restype = ctypes.c_size_t
    lib.sg_convert_static_bytes.argtypes = []
    lib.sg_mask_set.restype = ctypes.c_int
    lib.sg_mask_set.argtypes = [ctypes.c_int32, P(sg_mat), P(sg_mask), ctypes.c_void_p]
    lib.sg_convert.restype = ctypes.c_int
    lib.sg_convert.argtypes = [P(sg_semiring), P(sg_mat), ctypes.c_int32, vp, ctypes.c_size_t, P(sg_mat_out), P(i64), vp]
    _libs[path] = lib
    if _lib is None:
        _lib = lib
    return lib


def use_library(path: str):
    """Route every later call of this binding through the library at `path`
    (e.g. CHECK_LIB_PATH); returns the previously used library's path."""
    global _lib
    prev = getattr(_lib, "_name", LIB_PATH) if _lib is not None else LIB_PATH
    _lib = None
    load_library(path)
    _lib = _libs[path]
    return prev


def _check(status: int, where: str):
    if status != 0:
        detail = ""
        if status == -7 and _lib is not None:
            detail = (_lib.sg_last_error() or b"").decode(errors="replace")
        raise SgError(status, where, detail)


def _torch():
    import torch
    return torch


def _value_dtype(semiring: str):
    torch = _torch()
    return {"plus_times_f64": torch.float64, "plus_times_f32": torch.float32,
            "min_plus_i32": torch.int32, "or_and_bool": None}[semiring]


def default_tuning(semiring: str) -> sg_tuning:
    t = sg_tuning()
    load_library().sg_tuning_default(SEMIRINGS[semiring], ctypes.byref(t))
    return t


def make_tuning(semiring: str, **kw) -> sg_tuning:
    t = default_tuning(semiring)
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


class DevMat:
    """A sparse operand or result whose arrays are torch tensors on the GPU."""

    def __init__(self, fmt: str, nrows: int, ncols: int, ptr, idx, val=None, vid=None):
        self.fmt = fmt
        self.nrows = int(nrows)
        self.ncols = int(ncols)
        self.ptr = ptr
        self.idx = idx
        self.val = val
        self.vid = vid

    @property
    def nnz(self) -> int:
        return int(self.idx.numel())

    @property
    def nvec(self) -> int:
        return int(self.ptr.numel() - 1)

    @classmethod
    def from_host(cls, M, device="cuda", semiring: Optional[str] = None):
        """Copy a host matrix (numpy arrays: fmt, nrows, ncols, ptr, idx, val, vid) to the device."""
        torch = _torch()
        ptr = torch.as_tensor(np.ascontiguousarray(M.ptr, dtype=np.int64)).to(device)
        idx = torch.as_tensor(np.ascontiguousarray(M.idx, dtype=np.int32)).to(device)
        val = None
        if M.val is not None and semiring != "or_and_bool":
            val = torch.as_tensor(np.ascontiguousarray(M.val)).to(device)
        vid = None
        if M.fmt in ("dcsr", "dcsc"):
            vid = torch.as_tensor(np.ascontiguousarray(M.vid, dtype=np.int32)).to(device)
        return cls(M.fmt, M.nrows, M.ncols, ptr, idx, val, vid)

    def to_host(self):
        """numpy copy (a simple namespace with the same fields)."""
        import types
        return types.SimpleNamespace(
            fmt=self.fmt, nrows=self.nrows, ncols=self.ncols, ptr=self.ptr.cpu().numpy(),
            idx=self.idx.cpu().numpy(), val=None if self.val is None else self.val.cpu().numpy(),
            vid=None if self.vid is None else self.vid.cpu().numpy())

    def desc(self) -> sg_mat:
        d = sg_mat()
        d.fmt = FORMATS[self.fmt]
        d.nrows = self.nrows
        d.ncols = self.ncols
        d.nvec = self.nvec
        d.nnz = self.nnz
        d.ptr = self.ptr.data_ptr()
        d.vid = self.vid.data_ptr() if self.vid is not None and self.vid.numel() else None
        d.idx = self.idx.data_ptr() if self.idx.numel() else None
        d.val = self.val.data_ptr() if self.val is not None and self.val.numel() else None
        return d


class _nullctx:
    def __enter__(self):
        return None

    def __exit__(self, *a):
        return False


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A symbolic plan: the library handle, its workspace and the operands it refers to."""

    def __init__(self, semiring, As, Bs, group, ngroup, out_fmt, tuning, handle, ws, infos, stream=None):
        self.lib = load_library()  # the library that made the handle
        self.stream = stream
        self.semiring = semiring
        self.As, self.Bs = list(As), list(Bs)
        self.group = group
        self.ngroup = ngroup
        self.out_fmt = out_fmt
        self.tuning = tuning
        self.handle = handle
        self.ws = ws
        self.infos = infos

    def profile(self, enable: bool = True):
        """Record HIP events around every kernel launch of later numeric/batched calls."""
        _check(self.lib.sg_plan_profile(self.handle, 1 if enable else 0), "sg_plan_profile")

    def kernel_times(self):
        """Milliseconds of the last profiled call: heavy (or persistent), mid, tiny, pointers."""
        out = (ctypes.c_double * 4)()
        _check(self.lib.sg_plan_kernel_times(self.handle, out, 4), "sg_plan_kernel_times")
        return {"heavy": out[0], "mid": out[1], "tiny": out[2], "ptr": out[3]}

    def check(self):
        """Invariant counters of a checking build: (LDS left dirty, count mismatches)."""
        out = (ctypes.c_int64 * 2)()
        _check(self.lib.sg_plan_check(self.handle, out, 2), "sg_plan_check")
        return int(out[0]), int(out[1])

    def destroy(self):
        """Release the handle (host only, never waits for the device). The workspace
        tensor stays referenced by this object until it is garbage collected; it was
        allocated on the plan's stream, so the caching allocator hands it out again
        only in that stream's order."""
        if self.handle:
            self.lib.sg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def out_shapes(self):
        shapes = []
        for g in range(self.ngroup):
            p = self.group.index(g) if self.group is not None else g
            shapes.append((self.As[p].nrows, self.Bs[p].ncols))
        return shapes

    def alloc_outputs(self, device="cuda") -> List[DevMat]:
        """Exactly sized output matrices (torch allocations on the plan's stream) for every group."""
        torch = _torch()
        with torch.cuda.stream(self.stream) if self.stream is not None else _nullctx():
            return self._alloc_outputs(device)

    def _alloc_outputs(self, device):
        torch = _torch()
        vdt = _value_dtype(self.semiring)
        outs = []
        for g, (m, n) in enumerate(self.out_shapes()):
            info = self.infos[g]
            nnz = info["nnz"]
            doubly = self.out_fmt in ("dcsr", "dcsc")
            nvec = info["nvec"]
            ptr = torch.empty(nvec + 1, dtype=torch.int64, device=device)
            vid = torch.empty(nvec, dtype=torch.int32, device=device) if doubly else None
            idx = torch.empty(nnz, dtype=torch.int32, device=device)
            val = torch.empty(nnz, dtype=vdt, device=device) if vdt is not None else None
            outs.append(DevMat(self.out_fmt, m, n, ptr, idx, val, vid))
        return outs


def _out_descs(Cs: Sequence[DevMat]):
    arr = (sg_mat_out * len(Cs))()
    for i, C in enumerate(Cs):
        d = arr[i]
        d.fmt = FORMATS[C.fmt]
        d.nrows = C.nrows
        d.ncols = C.ncols
        d.cap_nnz = C.idx.numel()
        d.cap_vec = C.vid.numel() if C.vid is not None else 0
        d.ptr = C.ptr.data_ptr()
        d.vid = C.vid.data_ptr() if C.vid is not None and C.vid.numel() else None
        d.idx = C.idx.data_ptr() if C.idx.numel() else None
        d.val = C.val.data_ptr() if C.val is not None and C.val.numel() else None
    return arr


def _descs(Ms: Sequence[DevMat]):
    arr = (sg_mat * len(Ms))()
    for i, M in enumerate(Ms):
        arr[i] = M.desc()
    return arr


def workspace_size(semiring, As, Bs, group=None, ngroup=None, out_fmt=None, tuning=None) -> int:
    lib = load_library()
    sr = sg_semiring(SEMIRINGS[semiring])
    out_fmt = out_fmt or As[0].fmt
    A = _descs(As)
    B = _descs(Bs)
    g, ng = _groups(group, ngroup, len(As))
    sz = ctypes.c_size_t(0)
    _check(lib.sg_spgemm_workspace_size(ctypes.byref(sr), len(As), A, B, g, ng, FORMATS[out_fmt],
                                        ctypes.byref(tuning) if tuning is not None else None, ctypes.byref(sz)),
           "sg_spgemm_workspace_size")
    return int(sz.value)


def _groups(group, ngroup, nprod):
    if group is None:
        return None, nprod
    arr = (ctypes.c_int32 * nprod)(*[int(x) for x in group])
    return ctypes.cast(arr, ctypes.c_void_p), int(ngroup if ngroup is not None else max(group) + 1)


class Mask:
    """An output mask: a device int32/uint32 tensor of stride_words words per output
    vector (bit i % 32 of word [j, i / 32] for output id i of vector j);
    complement=True keeps the entries whose bit is clear."""

    def __init__(self, bits, stride_words: int, complement: bool = True):
        self.bits, self.stride_words, self.complement = bits, int(stride_words), bool(complement)

    @classmethod
    def zeros(cls, nvec: int, minor: int, device="cuda", complement: bool = True) -> "Mask":
        torch = _torch()
        stride = (int(minor) + 31) // 32
        return cls(torch.zeros(int(nvec) * stride, dtype=torch.int32, device=device), stride, complement)

    def desc(self) -> sg_mask:
        return sg_mask(self.bits.data_ptr(), self.stride_words, 1 if self.complement else 0, 0)


def mask_set(Ms: Sequence[DevMat], masks: Sequence[Mask], stream=None):
    """Set the bits of every stored entry of Ms[k] in masks[k] (on the device)."""
    if not Ms:
        return
    arr = _descs(Ms)
    marr = (sg_mask * len(masks))(*[m.desc() for m in masks])
    _check(load_library().sg_mask_set(len(Ms), arr, marr, _stream(stream)), "sg_mask_set")


def spgemm_symbolic(semiring: str, As: Sequence[DevMat], Bs: Sequence[DevMat], group=None, ngroup=None,
                    out_fmt: Optional[str] = None, tuning: Optional[sg_tuning] = None, stream=None,
                    ws=None, masks: Optional[Sequence[Optional[Mask]]] = None) -> Plan:
    """Symbolic phase (sizes, tiers, exact counts) of C_g = sum over group g of A_p B_p
    (with masks[g] applied to C_g when given)."""
    torch = _torch()
    lib = load_library()
    sr = sg_semiring(SEMIRINGS[semiring])
    out_fmt = out_fmt or As[0].fmt
    A = _descs(As)
    B = _descs(Bs)
    garr, ng = _groups(group, ngroup, len(As))
    sz = ctypes.c_size_t(0)
    tptr = ctypes.byref(tuning) if tuning is not None else None
    _check(lib.sg_spgemm_workspace_size(ctypes.byref(sr), len(As), A, B, garr, ng, FORMATS[out_fmt], tptr,
                                        ctypes.byref(sz)), "sg_spgemm_workspace_size")
    if ws is None or ws.numel() < sz.value:
        # allocated on the stream the kernels run on, so the caching allocator
        # reuses it only in that stream's order after the plan is dropped
        with torch.cuda.stream(stream) if stream is not None else _nullctx():
            ws = torch.empty(int(sz.value), dtype=torch.uint8, device=As[0].ptr.device)
    handle = ctypes.c_void_p(0)
    infos = (sg_sym_info * ng)()
    if masks is None:
        _check(lib.sg_spgemm_symbolic(ctypes.byref(sr), len(As), A, B, garr, ng, FORMATS[out_fmt], tptr,
                                      ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                      ctypes.byref(handle), infos, _stream(stream)), "sg_spgemm_symbolic")
    else:
        marr = (sg_mask * ng)(*[(m.desc() if m is not None else sg_mask(None, 0, 0, 0)) for m in masks])
        _check(lib.sg_spgemm_symbolic_masked(ctypes.byref(sr), len(As), A, B, garr, ng, FORMATS[out_fmt], marr, tptr,
                                             ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                             ctypes.byref(handle), infos, _stream(stream)),
               "sg_spgemm_symbolic_masked")
    glist = None if group is None else [int(x) for x in group]
    return Plan(semiring, As, Bs, glist, ng, out_fmt, tuning, handle, ws, [infos[i].as_dict() for i in range(ng)],
                stream)


def spgemm_numeric(plan: Plan, Cs: Sequence[DevMat], stream=None):
    arr = _out_descs(Cs)
    _check(plan.lib.sg_spgemm_numeric(plan.handle, arr, _stream(stream)), "sg_spgemm_numeric")


def spgemm_batched(plan: Plan, Cs: Sequence[DevMat], stream=None):
    arr = _out_descs(Cs)
    _check(plan.lib.sg_spgemm_batched(plan.handle, arr, _stream(stream)), "sg_spgemm_batched")


def spgemm(semiring: str, A: DevMat, B: DevMat, out_fmt: Optional[str] = None, tuning=None, batched=False,
           stream=None) -> DevMat:
    """C = A (x) B in one call (symbolic, allocation, numeric)."""
    plan = spgemm_symbolic(semiring, [A], [B], out_fmt=out_fmt, tuning=tuning, stream=stream)
    C = plan.alloc_outputs(A.ptr.device)  # on the plan's stream
    (spgemm_batched if batched else spgemm_numeric)(plan, C, stream)
    plan.destroy()
    return C[0]


def spgemm_grouped(semiring: str, As, Bs, group, ngroup, out_fmt=None, tuning=None, batched=True, stream=None):
    """C_g = (+) over p with group[p] = g of A_p (x) B_p, every product in one plan."""
    plan = spgemm_symbolic(semiring, As, Bs, group, ngroup, out_fmt=out_fmt, tuning=tuning, stream=stream)
    C = plan.alloc_outputs(As[0].ptr.device)
    (spgemm_batched if batched else spgemm_numeric)(plan, C, stream)
    plan.destroy()
    return C


def validate(M: DevMat, stream=None) -> bool:
    torch = _torch()
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        ws = torch.empty(64, dtype=torch.uint8, device=M.ptr.device)  # on the stream the check runs on
    d = M.desc()
    st = load_library().sg_validate(ctypes.byref(d), ctypes.c_void_p(ws.data_ptr()), _stream(stream))
    if st == -3:
        return False
    _check(st, "sg_validate")
    return True


def build_aux(M: DevMat, stream=None):
    """AUX column index of a doubly compressed matrix (device int32 tensor)."""
    torch = _torch()
    maj = M.nrows if M.fmt == "dcsr" else M.ncols
    nvec = M.nvec
    chunk = -(-maj // nvec) if nvec > 0 else max(maj, 1)
    chunk = max(chunk, 1)
    nchunks = -(-maj // chunk)
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        aux = torch.empty(nchunks + 1, dtype=torch.int32, device=M.ptr.device)  # on the stream that fills it
    n = ctypes.c_int64(0)
    d = M.desc()
    _check(load_library().sg_build_aux(ctypes.byref(d), ctypes.c_void_p(aux.data_ptr()), ctypes.byref(n),
                                       _stream(stream)), "sg_build_aux")
    assert n.value == nchunks
    return aux


def _new_mat(semiring, fmt, nrows, ncols, nnz, nvec, device):
    torch = _torch()
    vdt = _value_dtype(semiring)
    major = nrows if fmt in ("csr", "dcsr") else ncols
    doubly = fmt in ("dcsr", "dcsc")
    ptr = torch.empty((nvec if doubly else major) + 1, dtype=torch.int64, device=device)
    vid = torch.empty(nvec, dtype=torch.int32, device=device) if doubly else None
    idx = torch.empty(nnz, dtype=torch.int32, device=device)
    val = torch.empty(nnz, dtype=vdt, device=device) if vdt is not None else None
    return DevMat(fmt, nrows, ncols, ptr, idx, val, vid)


def coo_to_sparse(semiring: str, rows, cols, vals, nrows: int, ncols: int, fmt: str, stream=None) -> DevMat:
    """Canonical `fmt` matrix of device triples (int32 rows/cols, values or None), built on
    the device; repeated positions are combined with the semiring's add in list order."""
    torch = _torch()
    lib = load_library()
    sr = sg_semiring(SEMIRINGS[semiring])
    n = int(rows.numel())
    sz = ctypes.c_size_t(0)
    _check(lib.sg_coo_workspace_size(ctypes.byref(sr), nrows, ncols, n, FORMATS[fmt], ctypes.byref(sz)),
           "sg_coo_workspace_size")
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        ws = torch.empty(int(sz.value), dtype=torch.uint8, device=rows.device)
    nnz, nvec = ctypes.c_int64(0), ctypes.c_int64(0)
    vptr = vals.data_ptr() if vals is not None and vals.numel() else None
    _check(lib.sg_coo_compress(ctypes.byref(sr), nrows, ncols, n, rows.data_ptr() if n else None,
                               cols.data_ptr() if n else None, vptr, FORMATS[fmt], ws.data_ptr(), ws.numel(),
                               ctypes.byref(nnz), ctypes.byref(nvec), _stream(stream)), "sg_coo_compress")
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        M = _new_mat(semiring, fmt, nrows, ncols, int(nnz.value), int(nvec.value), rows.device)
    out = _out_descs([M])
    _check(lib.sg_coo_emit(ctypes.byref(sr), nrows, ncols, n, FORMATS[fmt], ws.data_ptr(), ws.numel(), nnz.value,
                           nvec.value, out, _stream(stream)), "sg_coo_emit")
    M._keep = ws  # the workspace is released with the matrix (stream-ordered reuse)
    return M


def convert(semiring: str, M: DevMat, fmt: str, stream=None) -> DevMat:
    """M in another format (device): the transpose of the storage between orientations."""
    torch = _torch()
    lib = load_library()
    sr = sg_semiring(SEMIRINGS[semiring])
    d = M.desc()
    sz = ctypes.c_size_t(0)
    _check(lib.sg_convert_workspace_size(ctypes.byref(sr), ctypes.byref(d), FORMATS[fmt], ctypes.byref(sz)),
           "sg_convert_workspace_size")
    major = M.nrows if fmt in ("csr", "dcsr") else M.ncols
    cap_vec = min(M.nnz, major) if fmt in ("dcsr", "dcsc") else 0
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        ws = torch.empty(int(sz.value), dtype=torch.uint8, device=M.ptr.device)
        out = _new_mat(semiring, fmt, M.nrows, M.ncols, M.nnz, cap_vec, M.ptr.device)
    desc = _out_descs([out])
    nv = ctypes.c_int64(0)
    _check(lib.sg_convert(ctypes.byref(sr), ctypes.byref(d), FORMATS[fmt], ws.data_ptr(), ws.numel(), desc,
                          ctypes.byref(nv), _stream(stream)), "sg_convert")
    if fmt in ("dcsr", "dcsc"):
        out.vid = out.vid[: nv.value]
        out.ptr = out.ptr[: nv.value + 1]
    out._keep = ws
    return out


def chain_symbolic(semiring: str, Xs: Sequence[DevMat], Ys: Sequence[DevMat], Zs: Sequence[DevMat],
                   out_fmt: Optional[str] = None, tuning: Optional[sg_tuning] = None, stream=None) -> Plan:
    """Plan of the fused chains C_p = X_p Y_p Z_p (one output per chain): the
    intermediate products are never written. Numeric calls as for any plan."""
    torch = _torch()
    lib = load_library()
    sr = sg_semiring(SEMIRINGS[semiring])
    out_fmt = out_fmt or Xs[0].fmt
    X, Y, Z = _descs(Xs), _descs(Ys), _descs(Zs)
    n = len(Xs)
    sz = ctypes.c_size_t(0)
    tptr = ctypes.byref(tuning) if tuning is not None else None
    _check(lib.sg_chain_workspace_size(ctypes.byref(sr), n, X, Y, Z, FORMATS[out_fmt], tptr, ctypes.byref(sz)),
           "sg_chain_workspace_size")
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        ws = torch.empty(int(sz.value), dtype=torch.uint8, device=Xs[0].ptr.device)
    handle = ctypes.c_void_p(0)
    infos = (sg_sym_info * n)()
    _check(lib.sg_chain_symbolic(ctypes.byref(sr), n, X, Y, Z, FORMATS[out_fmt], tptr, ctypes.c_void_p(ws.data_ptr()),
                                 ctypes.c_size_t(ws.numel()), ctypes.byref(handle), infos, _stream(stream)),
           "sg_chain_symbolic")
    plan = Plan(semiring, list(Xs), list(Zs), None, n, out_fmt, tuning, handle, ws, [infos[i].as_dict() for i in range(n)],
                stream)
    plan.operands = (list(Xs), list(Ys), list(Zs))  # the plan refers to all three
    return plan


def convert_into(semiring: str, M: DevMat, out: DevMat, static: bool = False, stream=None) -> int:
    """M in the format of the caller-allocated `out` (capacities: M's entries; doubly
    compressed output at least min(nnz, major) vectors). static=True uses the
    library's fixed workspace (sg_convert_static: no allocation at all); otherwise a
    workspace tensor is allocated. Returns the output's stored vectors."""
    torch = _torch()
    lib = load_library()
    sr = sg_semiring(SEMIRINGS[semiring])
    d = M.desc()
    desc = _out_descs([out])
    nv = ctypes.c_int64(0)
    if static:
        _check(lib.sg_convert_static(ctypes.byref(sr), ctypes.byref(d), FORMATS[out.fmt], desc, ctypes.byref(nv),
                                     _stream(stream)), "sg_convert_static")
        return int(nv.value)
    sz = ctypes.c_size_t(0)
    _check(lib.sg_convert_workspace_size(ctypes.byref(sr), ctypes.byref(d), FORMATS[out.fmt], ctypes.byref(sz)),
           "sg_convert_workspace_size")
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        ws = torch.empty(int(sz.value), dtype=torch.uint8, device=M.ptr.device)
    _check(lib.sg_convert(ctypes.byref(sr), ctypes.byref(d), FORMATS[out.fmt], ws.data_ptr(), ws.numel(), desc,
                          ctypes.byref(nv), _stream(stream)), "sg_convert")
    out._keep = ws
    return int(nv.value)


TUNE_FORMS = {"numeric": 0, "batched": 1, "numeric_reuse": 2}


def autotune_native(semiring: str, As: Sequence[DevMat], Bs: Sequence[DevMat], group=None, ngroup=None,
                    out_fmt: Optional[str] = None, form: str = "numeric", reps: int = 3, tuning=None, stream=None):
    """The library's own search (sg_autotune): returns (sg_tuning, best_ms, start_ms).
    form as in autotune.autotune: "numeric", "batched" or "numeric_reuse"."""
    lib = load_library()
    sr = sg_semiring(SEMIRINGS[semiring])
    group, ngroup = _groups(group, ngroup, len(As))
    out_fmt = out_fmt or As[0].fmt
    t = tuning if tuning is not None else default_tuning(semiring)
    t = sg_tuning.from_buffer_copy(t)
    a, b = _descs(As), _descs(Bs)
    best, start = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib.sg_autotune(ctypes.byref(sr), len(As), a, b, group, ngroup, FORMATS[out_fmt], TUNE_FORMS[form], reps,
                           ctypes.byref(t), ctypes.byref(best), ctypes.byref(start), _stream(stream)), "sg_autotune")
    return t, best.value, start.value
