"""The allocation-free entry point sg_convert_static (through the C ABI): the
same results as sg_convert with a caller workspace, on two calls in a row (the
second with a smaller input, so it runs on the array the first one left
behind), and a clear refusal of an input beyond the fixed workspace."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _outputs(sg, semiring, M, fmt):
    import torch
    major = M.nrows if fmt in ("csr", "dcsr") else M.ncols
    doubly = fmt in ("dcsr", "dcsc")
    nvec = min(M.nnz, major) if doubly else major
    vdt = {"plus_times_f64": torch.float64, "min_plus_i32": torch.int32, "or_and_bool": None}[semiring]
    mk = lambda: sg.DevMat(fmt, M.nrows, M.ncols, torch.full((nvec + 1,), -7, dtype=torch.int64, device="cuda"),
                           torch.full((M.nnz,), -7, dtype=torch.int32, device="cuda"),
                           None if vdt is None else torch.full((M.nnz,), 7, dtype=vdt, device="cuda"),
                           torch.full((nvec,), -7, dtype=torch.int32, device="cuda") if doubly else None)
    return mk(), mk()


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32", "or_and_bool"])
def test_convert_static_equals_convert(semiring):
    import torch
    import paper_1006_2183_amd as sg
    from paper_1006_2183_amd import binding
    binding.load_library()
    for scale, fmt in ((13, "csc"), (10, "dcsc"), (12, "csr"), (9, "dcsr")):  # each call smaller or different
        A = W.rmat_matrix(scale, 8, semiring, "csr", seed=scale)
        src = W.to_format(A, "csr" if fmt in ("csc", "dcsc") else "csc", semiring)
        dM = sg.DevMat.from_host(src, "cuda", semiring)
        a, b = _outputs(sg, semiring, src, fmt)
        na = binding.convert_into(semiring, dM, a, static=True)
        nb = binding.convert_into(semiring, dM, b, static=False)
        torch.cuda.synchronize()
        assert na == nb
        assert torch.equal(a.ptr[: na + 1 if fmt.startswith("d") else a.ptr.numel()],
                           b.ptr[: nb + 1 if fmt.startswith("d") else b.ptr.numel()])
        assert torch.equal(a.idx, b.idx)
        if a.val is not None:
            assert torch.equal(a.val, b.val)
        if a.vid is not None:
            assert torch.equal(a.vid[:na], b.vid[:nb])


def test_convert_static_refuses_beyond_its_workspace():
    import torch
    import paper_1006_2183_amd as sg
    from paper_1006_2183_amd import binding
    lib = binding.load_library()
    cap = int(lib.sg_convert_static_bytes())
    # a descriptor of a matrix whose workspace would exceed the array (no device data is read)
    n = cap // 8
    ptr = torch.zeros(2, dtype=torch.int64, device="cuda")
    idx = torch.zeros(1, dtype=torch.int32, device="cuda")
    val = torch.zeros(1, dtype=torch.float64, device="cuda")
    M = sg.DevMat("csr", 1, 1 << 20, ptr, idx, val)
    d = M.desc()
    d.nnz = n  # claims n entries: refused on the size alone, before any launch
    out = binding._out_descs([sg.DevMat("csc", 1, 1 << 20, torch.zeros((1 << 20) + 1, dtype=torch.int64, device="cuda"),
                                        idx, val)])
    nv = binding.ctypes.c_int64(0)
    st = lib.sg_convert_static(binding.ctypes.byref(binding.sg_semiring(0)), binding.ctypes.byref(d), 1, out,
                               binding.ctypes.byref(nv), None)
    assert st == -5
    assert b"static workspace" in lib.sg_last_error()
