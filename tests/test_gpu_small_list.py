"""The mid tier's one-wavefront form (the small list) on crafted vectors: runs
of equal ids that span lanes and registers, a whole vector on one id, exactly
1024 products (all sixteen registers), distinct ids, a vector one product over
the bound (which must take another tier), and the id-range bound of the packed
sort keys. Every case is compared with the oracle; force_tier 3 sends every
vector of at most 1024 products to the small list whatever the plan's size."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import assert_canonical, assert_same

pytestmark = pytest.mark.gpu

SEMIRINGS = ["plus_times_f64", "plus_times_f32", "min_plus_i32", "or_and_bool"]


def _say(msg):
    print(f"[small-list] {msg}", flush=True)


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1006_2183_amd as sg
    sg.load_library()
    return sg


def _vals(rng, n, semiring):
    if semiring == "or_and_bool":
        return None
    if semiring == "min_plus_i32":
        return rng.integers(0, 100, n).astype(np.int32)
    v = rng.uniform(0.5, 1.5, n)
    return v.astype(np.float32) if semiring == "plus_times_f32" else v


def crafted(semiring, nrows=4096, top=False, seed=11):
    """A (nrows x 2048, gathered) and B (2048 x 8, streamed), column-major, so
    that C(:, j) takes products of B(:, j)'s entries with A's columns:
      j=0: 1000 products, all on one id (a run over every lane and register);
      j=1: 32 x 32 = 1024 products on overlapping id ranges (runs of two);
      j=2: 33 x 32 = 1056 products (over the bound: another tier);
      j=3: 100 x 10 products on 70 ids (runs of about 14, across lanes);
      j=4: 70 products, distinct ids (two registers per lane);
      j=5: empty;
      j=6: 65 products, distinct ids;
      j=7: 32 x 32 = 1024 products, all distinct ids.
    top=True shifts every id to the top of the id range."""
    rng = np.random.default_rng(seed)
    ar, ac = [], []
    br, bc = [], []
    off = nrows - 2048 if top else 0

    def acol(k, ids):
        ar.extend(int(i) + off for i in ids)
        ac.extend([k] * len(ids))

    def bcol(j, ks):
        br.extend(ks)
        bc.extend([j] * len(ks))

    for k in range(1000):
        acol(k, [5])
    bcol(0, list(range(1000)))
    for t in range(32):
        acol(1000 + t, range(t * 16, t * 16 + 32))
    bcol(1, list(range(1000, 1032)))
    for t in range(33):
        acol(1032 + t, range(600 + t * 16, 600 + t * 16 + 32))
    bcol(2, list(range(1032, 1065)))
    for t in range(100):
        acol(1100 + t, [1200 + (t % 7) * 3 + 60 * q for q in range(10) if 1200 + (t % 7) * 3 + 60 * q < 2048][:10])
    bcol(3, list(range(1100, 1200)))
    acol(1300, range(1300, 1370))
    bcol(4, [1300])
    acol(1400, range(1400, 1465))
    bcol(6, [1400])
    for t in range(32):
        acol(1500 + t, range(t * 32, t * 32 + 32))
    bcol(7, list(range(1500, 1532)))
    A = W.from_triples(np.array(ar), np.array(ac), _vals(rng, len(ar), semiring), nrows, 2048, "csc", semiring)
    B = W.from_triples(np.array(br), np.array(bc), _vals(rng, len(br), semiring), 2048, 8, "csc", semiring)
    return A, B


def _run(sg, semiring, A, B, batched, **tune):
    import torch
    dA = sg.DevMat.from_host(A, "cuda", semiring)
    dB = sg.DevMat.from_host(B, "cuda", semiring)
    plan = sg.spgemm_symbolic(semiring, [dA], [dB], out_fmt="csc", tuning=sg.make_tuning(semiring, **tune))
    C = plan.alloc_outputs()
    (sg.spgemm_batched if batched else sg.spgemm_numeric)(plan, C)
    torch.cuda.synchronize()
    info = plan.infos[0]
    plan.destroy()
    return C[0].to_host(), info


def _rtol(semiring):
    return {"plus_times_f64": 1e-12, "plus_times_f32": 1e-5}.get(semiring, 0.0)


@pytest.mark.parametrize("semiring", SEMIRINGS)
@pytest.mark.parametrize("batched", [False, True])
def test_small_list_crafted_vectors(sg, semiring, batched):
    _say(f"case crafted {semiring} batched={batched}")
    A, B = crafted(semiring)
    R, _ = oracle.spgemm(semiring, A, B)
    C, info = _run(sg, semiring, A, B, batched, force_tier=3)
    assert info["n_small"] == 6, info  # every non-empty column but the one over the bound
    assert_canonical(C)
    assert_same(C, R, semiring, _rtol(semiring), f"small list {semiring}")
    # the same product with the small list off: the workgroup tiers agree with it
    C0, info0 = _run(sg, semiring, A, B, batched, small_max_flops=0)
    assert info0["n_small"] == 0
    assert_same(C0, R, semiring, _rtol(semiring), f"small list off {semiring}")


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32"])
def test_small_list_id_range_bound(sg, semiring):
    """Ids up to 2^22 - 2 pack into sort keys below the padding key; an id range
    of 2^22 keeps the workgroup tiers."""
    for nrows, small in (((1 << 22) - 1, True), (1 << 22, False)):
        _say(f"case id range {nrows} {semiring}")
        A, B = crafted(semiring, nrows=nrows, top=True)
        R, _ = oracle.spgemm(semiring, A, B)
        C, info = _run(sg, semiring, A, B, True, force_tier=3)
        assert (info["n_small"] > 0) == small, (nrows, info["n_small"])
        assert_canonical(C)
        assert_same(C, R, semiring, _rtol(semiring), f"id range {nrows}")
