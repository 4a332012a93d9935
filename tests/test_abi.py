"""Host-only checks of the C ABI: the library loads, exports every declared
entry point, and the pure-host calls (defaults, status strings, workspace
sizing and argument checks) behave as the header states. No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sg_spgemm.h")


def _lib():
    from paper_1006_2183_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return binding.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = _lib()
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), f"{n} not exported"
    from paper_1006_2183_amd import binding
    assert sorted(binding.EXPORTS) == names


def test_status_strings_and_defaults():
    lib = _lib()
    assert lib.sg_status_string(0) == b"ok"
    assert lib.sg_status_string(-6) == b"output capacity too small"
    from paper_1006_2183_amd import binding
    for s in binding.SEMIRINGS:
        t = binding.default_tuning(s)
        assert 1 <= t.tiny_max_flops <= 64
        assert t.block_threads % 64 == 0
        assert 4096 <= t.lds_bytes <= 160 * 1024
        assert t.heavy_threads % 64 == 0 and 64 <= t.heavy_threads <= 1024
        assert 4096 <= t.heavy_lds_bytes <= 160 * 1024
        assert 0 <= t.small_max_flops <= 1024


def _fake(fmt, nrows, ncols, nvec, nnz, with_val=True):
    d = __import__("paper_1006_2183_amd.binding", fromlist=["sg_mat"]).sg_mat()
    d.fmt = {"csr": 0, "csc": 1, "dcsr": 2, "dcsc": 3}[fmt]
    d.nrows, d.ncols, d.nvec, d.nnz = nrows, ncols, nvec, nnz
    # host-only calls never dereference these
    d.ptr = 0x1000
    d.idx = 0x2000 if nnz else None
    d.val = 0x3000 if with_val else None
    d.vid = 0x4000 if fmt in ("dcsr", "dcsc") else None
    return d


def _wsize(lib, kind, A, B, out_fmt, group=None, ngroup=None):
    from paper_1006_2183_amd import binding
    sr = binding.sg_semiring(kind)
    n = len(A)
    Aa = (binding.sg_mat * n)(*A)
    Ba = (binding.sg_mat * n)(*B)
    g = None
    if group is not None:
        g = ctypes.cast((ctypes.c_int32 * n)(*group), ctypes.c_void_p)
    sz = ctypes.c_size_t(0)
    st = lib.sg_spgemm_workspace_size(ctypes.byref(sr), n, Aa, Ba, g, ngroup or n, out_fmt, None, ctypes.byref(sz))
    return st, sz.value


def test_workspace_size_and_argument_checks():
    lib = _lib()
    A = _fake("csr", 100, 80, 100, 500)
    B = _fake("csr", 80, 60, 80, 400)
    st, sz = _wsize(lib, 0, [A], [B], 0)
    assert st == 0 and sz > 0
    # inner dimensions differ
    Bbad = _fake("csr", 81, 60, 81, 400)
    assert _wsize(lib, 0, [A], [Bbad], 0)[0] == -2
    # mixed orientation is unsupported
    Bcsc = _fake("csc", 80, 60, 60, 400)
    assert _wsize(lib, 0, [A], [Bcsc], 0)[0] == -4
    # output orientation must match
    assert _wsize(lib, 0, [A], [B], 1)[0] == -4
    # bad semiring / format
    assert _wsize(lib, 9, [A], [B], 0)[0] == -1
    # missing values for a valued semiring, allowed for boolean
    Anv = _fake("csr", 100, 80, 100, 500, with_val=False)
    assert _wsize(lib, 0, [Anv], [B], 0)[0] == -1
    assert _wsize(lib, 3, [Anv], [B], 0)[0] == 0
    # CSR must store one vector per row
    assert _wsize(lib, 0, [_fake("csr", 100, 80, 99, 500)], [B], 0)[0] == -1
    # groups: shapes inside a group must agree, and every group needs a product
    A2 = _fake("dcsc", 50, 40, 10, 30)
    B2 = _fake("dcsc", 40, 20, 5, 12)
    B3 = _fake("dcsc", 40, 21, 5, 12)
    assert _wsize(lib, 0, [A2, A2], [B2, B2], 3, group=[0, 0], ngroup=1)[0] == 0
    assert _wsize(lib, 0, [A2, A2], [B2, B3], 3, group=[0, 0], ngroup=1)[0] == -2
    assert _wsize(lib, 0, [A2], [B2], 3, group=[0], ngroup=2)[0] == -1
    # more products in one group do not shrink the workspace
    s1 = _wsize(lib, 0, [A2], [B2], 3)[1]
    s2 = _wsize(lib, 0, [A2] * 4, [B2] * 4, 3, group=[0] * 4, ngroup=1)[1]
    assert s2 >= s1


def test_binding_has_no_cpu_fallback():
    """The binding never imports the oracle and has no host compute path."""
    import paper_1006_2183_amd
    pkg = os.path.dirname(paper_1006_2183_amd.__file__)
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in src and "from oracle" not in src, f


def test_autotune_argument_checks():
    """sg_autotune refuses bad arguments before touching the device."""
    from paper_1006_2183_amd import binding
    lib = _lib()
    A = (binding.sg_mat * 1)(_fake("csr", 100, 80, 100, 500))
    B = (binding.sg_mat * 1)(_fake("csr", 80, 60, 80, 400))
    sr = binding.sg_semiring(0)
    t = binding.default_tuning("plus_times_f64")
    best, start = ctypes.c_double(0.0), ctypes.c_double(0.0)

    def call(form=0, reps=1, tuning=True, semiring=True):
        return lib.sg_autotune(ctypes.byref(sr) if semiring else None, 1, A, B, None, 1, 0, form, reps,
                               ctypes.byref(t) if tuning else None, ctypes.byref(best), ctypes.byref(start), None)
    assert call(form=3) == -1
    assert call(form=-1) == -1
    assert call(reps=0) == -1
    assert call(tuning=False) == -1
    assert call(semiring=False) == -1
