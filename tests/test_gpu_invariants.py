"""GPU runs of the invariant-checking build of the library (SG_CHECK=1).

The checking build computes the same results with the same kernels, and in
addition every persistent workgroup verifies after each work item that its
dynamic LDS is back to all-zero bits (the accumulators of every item kind
rely on starting from zero: heavy windows of both kinds, with and without
kept bitmaps or entry records, whole-range and hash mid vectors, tiny
chunks), and every numeric tier compares the number of entries it writes
for a vector or window with the exact count of the symbolic phase (the
entries one window writes must fill exactly the output range planned for
it, or neighbouring vectors overwrite each other in an order that depends
on scheduling). Each case asserts both counters are zero and the result
equals the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import assert_canonical, assert_same

pytestmark = pytest.mark.gpu

SEMIRINGS = ["plus_times_f64", "plus_times_f32", "min_plus_i32", "or_and_bool"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1006_2183_amd as sg
    from paper_1006_2183_amd import binding
    prev = binding.use_library(binding.CHECK_LIB_PATH)
    assert binding.load_library().sg_build_checked() == 1
    yield sg
    binding.use_library(prev)


def _run(sg, semiring, As, Bs, group=None, ngroup=None, out_fmt=None, batched=False, reps=1, **tune):
    import torch
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in As]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in Bs]
    t = sg.make_tuning(semiring, **tune) if tune else None
    plan = sg.spgemm_symbolic(semiring, dA, dB, group, ngroup, out_fmt=out_fmt, tuning=t)
    C = plan.alloc_outputs()
    for _ in range(reps):
        (sg.spgemm_batched if batched else sg.spgemm_numeric)(plan, C)
    torch.cuda.synchronize()
    lds, cnt = plan.check()
    plan.destroy()
    assert lds == 0, f"{lds} work items left LDS non-zero"
    assert cnt == 0, f"{cnt} numeric counts differ from the symbolic counts"
    return [c.to_host() for c in C]


def _oracle_check(semiring, C, A, B, what):
    R, _ = oracle.spgemm(semiring, A, B)
    assert_canonical(C)
    rtol = 1e-12 if semiring == "plus_times_f64" else (1e-4 if semiring == "plus_times_f32" else 0.0)
    if semiring == "plus_times_f32":
        assert_same(C, R, "or_and_bool", what=what)
        return
    assert_same(C, R, semiring, rtol, what)


@pytest.mark.parametrize("semiring", SEMIRINGS)
@pytest.mark.parametrize("batched", [False, True])
@pytest.mark.parametrize("cfg", [
    dict(),
    dict(lds_bytes=16384, block_threads=256, heavy_lds_bytes=16384, heavy_threads=256),
    dict(lds_bytes=16384, block_threads=256, heavy_lds_bytes=16384, heavy_threads=256, bitmap_mb=1),
    dict(lds_bytes=16384, block_threads=256, heavy_lds_bytes=16384, heavy_threads=256, bitmap_mb=0),
    dict(lds_bytes=16384, block_threads=256, heavy_lds_bytes=16384, heavy_threads=256, entry_mb=64),
    dict(lds_bytes=16384, block_threads=256, heavy_lds_bytes=16384, heavy_threads=256, mid_kind=1),
    dict(lds_bytes=16384, block_threads=256, heavy_lds_bytes=16384, heavy_threads=256, heavy_kind=1),
    dict(lds_bytes=8192, block_threads=128, heavy_lds_bytes=12288, heavy_threads=192, entry_mb=1),
    dict(lds_bytes=16384, block_threads=256, heavy_lds_bytes=16384, heavy_threads=256, force_tier=3, entry_mb=64),
    dict(small_max_flops=0),
])
def test_rmat_tiers_invariants(sg, semiring, batched, cfg):
    """All tiers in one launch (batched) or per tier, with small LDS budgets so that
    heavy vectors split into many windows and item kinds alternate on a workgroup."""
    _say(f"case invariants rmat s13 {semiring} batched={batched} {cfg}")
    A = W.rmat_matrix(13, 8, semiring, "csr", seed=4)
    (C,) = _run(sg, semiring, [A], [A], batched=batched, reps=2, **cfg)
    _oracle_check(semiring, C, A, A, f"{cfg}")


@pytest.mark.parametrize("batched", [False, True])
def test_summa_share_invariants(sg, batched):
    """A SUMMA share at scale 19 on a 16 x 16 grid (16 stage products of DCSC blocks
    accumulated into one output): fused, and with entry records."""
    sr = "plus_times_f64"
    grid, scale = 16, 19
    _say(f"case invariants SUMMA share s{scale} grid {grid} batched={batched}")
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (1, 2), semiring=sr, seed=7, fmt="dcsc")
    b = (1 << scale) // grid
    for tune in (dict(), dict(entry_mb=256), dict(lds_bytes=24576, heavy_lds_bytes=24576, heavy_threads=256),
                 dict(entry_mb=256, force_tier=3)):
        (C,) = _run(sg, sr, a_blocks, b_blocks, [0] * grid, 1, out_fmt="dcsc", batched=batched, reps=2, **tune)
        # oracle: the strips A(I, :) A(:, J)
        ra, ca, va, rb, cb, vb = [], [], [], [], [], []
        for k in range(grid):
            Ak, Bk = a_blocks[k], b_blocks[k]
            ra.append(Ak.idx.astype(np.int64)); va.append(Ak.val)
            ca.append(np.repeat(Ak.vid.astype(np.int64), np.diff(Ak.ptr)) + k * b)
            rb.append(Bk.idx.astype(np.int64) + k * b); vb.append(Bk.val)
            cb.append(np.repeat(Bk.vid.astype(np.int64), np.diff(Bk.ptr)))
        SA = W.from_triples(np.concatenate(ra), np.concatenate(ca), np.concatenate(va), b, grid * b, "dcsc", sr)
        SB = W.from_triples(np.concatenate(rb), np.concatenate(cb), np.concatenate(vb), grid * b, b, "dcsc", sr)
        _oracle_check(sr, C, SA, SB, f"summa {tune}")


def test_merge_and_galerkin_invariants(sg):
    """The partial-merge form (a grouped product with identity operands) and the
    grouped Galerkin products (many small instances, one output each)."""
    sr = "plus_times_f64"
    _say("case invariants merge + Galerkin")
    parts = [W.rmat_matrix(12, 8, sr, "dcsc", seed=30 + i) for i in range(8)]
    I = W.identity_matrix(parts[0].nrows, "csc", sr)
    (C,) = _run(sg, sr, [I] * 8, parts, [0] * 8, 1, out_fmt="dcsc", batched=True, reps=2)
    ref = parts[0]
    for p in parts[1:]:
        r1, c1, v1 = ref.triples()
        r2, c2, v2 = p.triples()
        ref = W.from_triples(np.concatenate([r1, r2]), np.concatenate([c1, c2]), np.concatenate([v1, v2]),
                             ref.nrows, ref.ncols, "dcsc", sr)
    assert_same(C, ref, sr, 1e-12, "merge")
    sizes = [8, 12, 16, 8, 24]
    Ls = [W.laplacian_7pt(n, "csr") for n in sizes]
    Ps = [W.aggregation_p(n, "csr") for n in sizes]
    APs = _run(sg, sr, Ls, Ps, list(range(len(sizes))), len(sizes), batched=True, reps=2)
    for i in range(len(sizes)):
        _oracle_check(sr, APs[i], Ls[i], Ps[i], f"AP {sizes[i]}")
