"""GPU parity of the masked products and the masked multi-level BFS built on
them (Section 6.2.2), through the C ABI:

* masked products against the oracle's product with the masked positions
  removed, for every semiring and tier (and both mask senses), in the
  invariant-checking build;
* the multi-source BFS, level by level, against the oracle's BFS (boolean,
  bit-exact), alone and served with iteration-level batching.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import bfs as OB
from oracle import convert as OC
from tests.helpers import assert_same

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1006_2183_amd as sg
    sg.load_library()
    return sg


def _masked_ref(semiring, A, B, bits, stride, complement):
    """Oracle product of column-major A B, then the entries whose mask bit says drop removed."""
    R, _ = oracle.spgemm(semiring, A, B)
    r, c, v = OC.triples(R)
    word = bits[c * stride + (r >> 5)]
    bit = (word >> (r & 31).astype(np.uint32)) & 1
    keep = bit == 0 if complement else bit == 1
    return W.from_triples(r[keep], c[keep], None if v is None else v[keep], R.nrows, R.ncols, "csc", semiring)


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32", "or_and_bool"])
@pytest.mark.parametrize("complement", [True, False])
@pytest.mark.parametrize("tune", [dict(), dict(force_tier=0), dict(force_tier=1), dict(force_tier=1, mid_kind=1),
                                  dict(force_tier=3), dict(small_max_flops=0),
                                  dict(force_tier=2, lds_bytes=16384, heavy_lds_bytes=16384, block_threads=256,
                                       heavy_threads=256),
                                  dict(force_tier=2, lds_bytes=16384, heavy_lds_bytes=16384, block_threads=256,
                                       heavy_threads=256, bitmap_mb=0),
                                  dict(force_tier=2, heavy_kind=1, lds_bytes=16384, heavy_lds_bytes=16384,
                                       block_threads=256, heavy_threads=256)])
def test_masked_product_every_tier(sg, semiring, complement, tune):
    import torch
    from paper_1006_2183_amd import binding
    _say(f"case masked {semiring} complement={complement} {tune}")
    prev = binding.use_library(binding.CHECK_LIB_PATH)
    try:
        A = W.rmat_matrix(12, 8, semiring, "csc", seed=6)
        Bm = W.to_format(W.rmat_matrix(12, 8, semiring, "csr", seed=7), "csc", semiring)
        n = A.nrows
        stride = (n + 31) // 32 + 3  # a padded stride
        rng = np.random.default_rng(1)
        bits = rng.integers(0, 2 ** 32, size=Bm.ncols * stride, dtype=np.uint64).astype(np.uint32)
        bits &= rng.integers(0, 2 ** 32, size=bits.size, dtype=np.uint64).astype(np.uint32)  # ~25% set
        dA = sg.DevMat.from_host(A, "cuda", semiring)
        dB = sg.DevMat.from_host(Bm, "cuda", semiring)
        mask = sg.Mask(torch.as_tensor(bits.view(np.int32)).cuda(), stride, complement)
        t = sg.make_tuning(semiring, **tune) if tune else None
        for batched in (False, True):
            plan = sg.spgemm_symbolic(semiring, [dA], [dB], tuning=t, masks=[mask])
            (C,) = plan.alloc_outputs()
            (sg.spgemm_batched if batched else sg.spgemm_numeric)(plan, [C])
            torch.cuda.synchronize()
            lds, cnt = plan.check()
            plan.destroy()
            assert lds == 0 and cnt == 0, (lds, cnt)
            ref = _masked_ref(semiring, A, Bm, bits, stride, complement)
            assert_same(C.to_host(), ref, semiring, 1e-12, f"masked batched={batched}")
    finally:
        binding.use_library(prev)


def test_masked_bfs_levels_match_oracle(sg):
    from paper_1006_2183_amd.bfs import MaskedBFS
    _say("case masked BFS rmat s14")
    A = W.rmat_matrix(14, 8, "or_and_bool", "csc", seed=21)
    dA = sg.DevMat.from_host(A, "cuda", "or_and_bool")
    rng = np.random.default_rng(4)
    src = rng.integers(0, A.nrows, 37)
    src[3] = src[5]  # the same source twice: two identical searches
    levels = MaskedBFS(dA).run(src)
    want = OB.bfs_levels(A, src)
    depth = max(len(w) for w in want)
    assert len(levels) == depth
    for d in range(depth):
        Y = levels[d].to_host()
        assert Y.ncols == len(src)
        for c in range(len(src)):
            exp = want[c][d] if d < len(want[c]) else np.zeros(0, np.int64)
            assert np.array_equal(Y.idx[Y.ptr[c]:Y.ptr[c + 1]], exp), f"level {d} column {c}"
    # a depth limit stops after that many levels
    assert len(MaskedBFS(dA).run(src, max_levels=2)) == min(3, depth)


@pytest.mark.parametrize("batched", [True, False])
def test_bfs_server_levels_match_oracle(sg, batched):
    from paper_1006_2183_amd.bfs import BfsRequest, BfsServer
    _say(f"case BFS server batched={batched}")
    A = W.rmat_matrix(13, 8, "or_and_bool", "csc", seed=22)
    dA = sg.DevMat.from_host(A, "cuda", "or_and_bool")
    rng = np.random.default_rng(9)
    arr = W.poisson_arrivals(3000.0, 24, 5)
    reqs = [BfsRequest(i, float(arr[i]), rng.integers(0, A.nrows, int(rng.integers(1, 40))),
                       int(rng.integers(1, 6))) for i in range(24)]
    srv = BfsServer(dA, pool_bytes=1 << 24, max_active=8, batched=batched)
    done = srv.run(reqs)
    assert all(r.status == "done" for r in done) and len(done) == 24
    if batched:
        assert any(len(m) > 1 for m in srv.mix), "no iteration mixed requests at different depths"
    for r in done:
        want = OB.bfs_levels(A, r.sources, max_levels=r.max_levels)
        got = [Y.to_host() for Y in r.levels]
        depth = max(len(w) for w in want)
        assert len(got) == depth, f"request {r.rid}"
        for d in range(depth):
            for c in range(len(r.sources)):
                exp = want[c][d] if d < len(want[c]) else np.zeros(0, np.int64)
                assert np.array_equal(got[d].idx[got[d].ptr[c]:got[d].ptr[c + 1]], exp), \
                    f"request {r.rid} level {d} column {c}"
