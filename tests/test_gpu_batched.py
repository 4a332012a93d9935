"""GPU parity of the batched forms: the Sparse SUMMA share (stage products
accumulated into one output), materialise-then-merge of stage partials,
uneven Galerkin R (A P) instances, and HIP-graph replays of the persistent
launch. Each is checked against the CPU oracle."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import assert_canonical, assert_same, triples

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


def strips(a_blocks, b_blocks, b, grid, semiring):
    """A(I, :) and A(:, J) as single doubly compressed operands (the oracle's reference)."""
    ra, ca, va, rb, cb, vb = [], [], [], [], [], []
    for k in range(grid):
        r, c, v = triples(a_blocks[k])
        ra.append(r); ca.append(c + k * b); va.append(v)
        r, c, v = triples(b_blocks[k])
        rb.append(r + k * b); cb.append(c); vb.append(v)
    cat = lambda x: None if x[0] is None else np.concatenate(x)
    SA = W.from_triples(np.concatenate(ra), np.concatenate(ca), cat(va), b, grid * b, "dcsc", semiring)
    SB = W.from_triples(np.concatenate(rb), np.concatenate(cb), cat(vb), grid * b, b, "dcsc", semiring)
    return SA, SB


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32", "or_and_bool"])
@pytest.mark.parametrize("batched", [False, True])
def test_summa_share_fused(sg, semiring, batched):
    """C_00 = (+)_k A_0k A_k0 over 8 stages (R-MAT scale 14 relabelled, 8 x 8 grid)."""
    from paper_1006_2183_amd import batched as BT
    _say(f"case summa share {semiring} batched={batched}")
    scale, grid = 14, 8
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (0, 0), semiring=semiring, seed=5)
    b = (1 << scale) // grid
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in b_blocks]
    C = BT.summa_share(semiring, dA, dB, batched=batched).to_host()
    SA, SB = strips(a_blocks, b_blocks, b, grid, semiring)
    R, flops = oracle.spgemm(semiring, SA, SB)
    assert_canonical(C)
    assert_same(C, R, semiring, 1e-12, "summa share")


def test_summa_share_forced_tiers_and_order(sg):
    """Every tier on the stage-merged output, and the stage order does not matter."""
    from paper_1006_2183_amd import batched as BT
    import torch
    semiring = "min_plus_i32"
    scale, grid = 13, 4
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (1, 2), semiring=semiring, seed=9)
    b = (1 << scale) // grid
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in b_blocks]
    SA, SB = strips(a_blocks, b_blocks, b, grid, semiring)
    R, _ = oracle.spgemm(semiring, SA, SB)
    for force in (-1, 1, 2, 3):
        t = sg.make_tuning(semiring, force_tier=force, lds_bytes=16384, block_threads=256, heavy_lds_bytes=16384,
                           heavy_threads=256)
        C = BT.summa_share(semiring, dA, dB, tuning=t).to_host()
        assert_same(C, R, semiring, 0.0, f"force {force}")
    perm = [3, 0, 2, 1]
    C = BT.summa_share(semiring, [dA[i] for i in perm], [dB[i] for i in perm]).to_host()
    assert_same(C, R, semiring, 0.0, "shuffled stages")
    torch.cuda.synchronize()


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32"])
def test_partials_then_merge(sg, semiring):
    """Materialised stage partials merged by a grouped identity product equal the fused share."""
    from paper_1006_2183_amd import batched as BT
    scale, grid = 13, 8
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (0, 0), semiring=semiring, seed=3)
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in b_blocks]
    partials = [sg.spgemm(semiring, a, bb, out_fmt="dcsc") for a, bb in zip(dA, dB)]
    for k in range(grid):
        Rk, _ = oracle.spgemm(semiring, a_blocks[k], b_blocks[k])
        assert_same(partials[k].to_host(), Rk, semiring, 1e-12, f"partial {k}")
    M = BT.merge_partials(semiring, partials).to_host()
    F = BT.summa_share(semiring, dA, dB).to_host()
    assert_canonical(M)
    assert_same(M, F, semiring, 1e-12, "merge vs fused")


def test_galerkin_uneven_instances(sg):
    """R (A P) = 4 L_{n/2} exactly, for 16 uneven 7-point grids in two grouped launches."""
    from paper_1006_2183_amd import batched as BT
    rng = np.random.default_rng(2)
    sizes = rng.choice([4, 6, 8, 10, 12], size=16)
    Ls = [W.laplacian_7pt(int(n), "csr") for n in sizes]
    Ps = [W.aggregation_p(int(n), "csr") for n in sizes]
    Rs = [W.transpose(P, "csr") for P in Ps]
    dev = lambda M: sg.DevMat.from_host(M, "cuda")
    for batched in (False, True):
        out = BT.galerkin_rap("plus_times_f64", [dev(R) for R in Rs], [dev(L) for L in Ls], [dev(P) for P in Ps],
                              batched=batched)
        for i, n in enumerate(sizes):
            Lc = W.laplacian_7pt(int(n) // 2, "csr")
            Lc.val = Lc.val * 4.0
            assert_same(out[i].to_host(), Lc, "plus_times_f64", 0.0, f"instance {i} n={n}")


def test_graph_replay_tracks_values(sg):
    """The persistent launch captured in a HIP graph: every replay equals an eager run on
    the current values, with eager work and synchronisations between replays."""
    import torch
    from paper_1006_2183_amd import batched as BT
    semiring = "plus_times_f64"
    scale, grid = 13, 4
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (0, 0), semiring=semiring, seed=11)
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in b_blocks]
    plan = BT.summa_share_plan(semiring, dA, dB)
    G = BT.GraphedNumeric(plan)
    scales = [1.0, 2.0, 0.5]
    for rep, f in enumerate(scales):
        for m in dA + dB:
            m.val.mul_(f)  # eager work between replays changes the operand values
        torch.cuda.synchronize()
        out = G.replay()[0]
        torch.cuda.synchronize()
        eager = plan.alloc_outputs()
        sg.spgemm_numeric(plan, eager)
        torch.cuda.synchronize()
        got = out.to_host()
        ref = eager[0].to_host()
        assert np.array_equal(got.ptr, ref.ptr) and np.array_equal(got.idx, ref.idx), f"replay {rep} pattern"
        assert np.allclose(got.val, ref.val, rtol=1e-12, atol=0), f"replay {rep} values"
        # and against the oracle on the current host values
        ha = [sg.DevMat.to_host(m) for m in dA]
        hb = [sg.DevMat.to_host(m) for m in dB]
        b = (1 << scale) // grid
        SA, SB = strips(ha, hb, b, grid, semiring)
        R, _ = oracle.spgemm(semiring, SA, SB)
        assert_same(got, R, semiring, 1e-12, f"replay {rep} vs oracle")
    plan.destroy()


@pytest.mark.parametrize("semiring", ["min_plus_i32", "or_and_bool"])
def test_integer_results_bitwise_reproducible(sg, semiring):
    """Integer and boolean semirings are exact, so every run of every form gives the same
    bytes: eager numeric runs, persistent launches, graph replays (records and the small
    list included), and the plain per-product path, equal to the oracle. (FP64 (+,*) is
    not bitwise reproducible: its LDS-atomic sums follow the schedule; its runs agree to
    the stated tolerance.)"""
    import torch
    from paper_1006_2183_amd import batched as BT
    _say(f"case integer reproducibility {semiring}")
    scale, grid = 15, 4  # 8192-wide blocks: the plan takes the small list too
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (0, 0), semiring=semiring, seed=21)
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in b_blocks]
    b = (1 << scale) // grid
    SA, SB = strips(a_blocks, b_blocks, b, grid, semiring)
    R, _ = oracle.spgemm(semiring, SA, SB)
    plan = BT.summa_share_plan(semiring, dA, dB, tuning=sg.make_tuning(semiring, entry_mb=64))
    assert plan.infos[0]["n_small"] > 0
    runs = []
    for _ in range(2):
        out = plan.alloc_outputs()
        sg.spgemm_numeric(plan, out)
        torch.cuda.synchronize()
        runs.append(out[0].to_host())
        out = plan.alloc_outputs()
        sg.spgemm_batched(plan, out)
        torch.cuda.synchronize()
        runs.append(out[0].to_host())
    G = BT.GraphedNumeric(plan)
    for _ in range(3):
        G.replay()
        torch.cuda.synchronize()
        runs.append(G.outputs[0].to_host())
    runs.append(BT.summa_share(semiring, dA, dB, batched=False).to_host())
    ref = runs[0]
    assert_same(ref, R, semiring, 0.0, "first run vs oracle")
    for i, c in enumerate(runs[1:]):
        assert np.array_equal(c.ptr, ref.ptr) and np.array_equal(c.idx, ref.idx), f"run {i + 1} pattern"
        assert np.array_equal(c.vid, ref.vid), f"run {i + 1} vector ids"
        if ref.val is not None:
            assert c.val.tobytes() == ref.val.tobytes(), f"run {i + 1} values"
    plan.destroy()


def test_galerkin_graph_chain_replay(sg):
    """A P then R (A P) captured in one graph: after scaling the operator by f,
    every replay gives R (f L_n) P = 4 f L_{n/2} exactly."""
    import torch
    from paper_1006_2183_amd import batched as BT
    sizes = [4, 8, 6, 12, 10, 8]
    Ls = [W.laplacian_7pt(n, "csr") for n in sizes]
    Ps = [W.aggregation_p(n, "csr") for n in sizes]
    Rs = [W.transpose(P, "csr") for P in Ps]
    dev = lambda M: sg.DevMat.from_host(M, "cuda")
    dL = [dev(L) for L in Ls]
    plan_ap, AP, plan_rap = BT.galerkin_plans("plus_times_f64", [dev(R) for R in Rs], dL, [dev(P) for P in Ps])
    G = BT.GraphedNumeric([plan_ap, plan_rap], [AP, None])
    total = 1.0
    for rep, f in enumerate([2.0, 0.5, 4.0]):
        for m in dL:
            m.val.mul_(f)
        total *= f
        torch.cuda.synchronize()
        out = G.replay()
        torch.cuda.synchronize()
        for i, n in enumerate(sizes):
            Lc = W.laplacian_7pt(n // 2, "csr")
            Lc.val = Lc.val * (4.0 * total)
            assert_same(out[i].to_host(), Lc, "plus_times_f64", 0.0, f"replay {rep} instance {i}")
    plan_ap.destroy()
    plan_rap.destroy()


def test_autotune_keeps_results(sg, tmp_path):
    """Every setting the tuner tries computes the same product; the cache round-trips."""
    import torch
    from paper_1006_2183_amd import autotune as AT
    semiring = "min_plus_i32"
    A = W.rmat_matrix(11, 16, semiring, "csr", seed=3)
    dA = sg.DevMat.from_host(A, "cuda", semiring)
    R, _ = oracle.spgemm(semiring, A, A)
    cache = AT.TuneCache(str(tmp_path / "tune.json"))
    space = {"lds_bytes": [16384, 65536], "heavy_lds_bytes": [24576], "blocks_per_cu": [1, 3], "tiny_max_flops": [16]}
    res = AT.autotune(semiring, [dA], [dA], space=space, reps=1, cache=cache)
    assert not res["cached"] and res["tried"] >= 2
    again = AT.autotune(semiring, [dA], [dA], space=space, reps=1, cache=AT.TuneCache(str(tmp_path / "tune.json")))
    assert again["cached"] and again["tuning"] == res["tuning"]
    t = AT.tuned(semiring, [dA], [dA], cache=cache)
    C = sg.spgemm(semiring, dA, dA, tuning=t).to_host()
    assert_same(C, R, semiring, 0.0, "tuned")
    for cand in ({"lds_bytes": 16384}, {"heavy_lds_bytes": 24576, "heavy_threads": 256},
                 {"blocks_per_cu": 3, "tiny_max_flops": 16}):
        C = sg.spgemm(semiring, dA, dA, tuning=sg.make_tuning(semiring, **cand)).to_host()
        assert_same(C, R, semiring, 0.0, str(cand))
    torch.cuda.synchronize()


@pytest.mark.parametrize("form", ["numeric", "batched", "numeric_reuse"])
def test_native_autotune(sg, form):
    """The library's own search (sg_autotune, through the C ABI): it returns a
    setting no slower than the one it started from, and that setting computes
    the oracle's product."""
    semiring = "plus_times_f64"
    _say(f"case native autotune {form}")
    A = W.rmat_matrix(11, 16, semiring, "csr", seed=3)
    dA = sg.DevMat.from_host(A, "cuda", semiring)
    R, _ = oracle.spgemm(semiring, A, A)
    t, best, start = sg.autotune_native(semiring, [dA], [dA], form=form, reps=1)
    assert 0.0 < best <= start
    C = sg.spgemm(semiring, dA, dA, tuning=t, batched=form != "numeric").to_host()
    assert_same(C, R, semiring, 1e-12, f"native autotune {form}")


def test_autotune_replay_presets_keep_results(sg):
    """The replayed-form search (presets first, then the record budget and tier
    thresholds) on a small SUMMA share: the chosen setting computes the
    oracle's result, and every preset and space value is a setting the
    library accepts for this plan."""
    from paper_1006_2183_amd import autotune as AT
    from paper_1006_2183_amd import batched as BT
    semiring = "plus_times_f64"
    scale, grid = 11, 8
    _say("case autotune replay presets")
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (1, 2), semiring=semiring, seed=5)
    b = (1 << scale) // grid
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in b_blocks]
    SA, SB = strips(a_blocks, b_blocks, b, grid, semiring)
    R, _ = oracle.spgemm(semiring, SA, SB)
    res = AT.autotune(semiring, dA, dB, [0] * grid, 1, out_fmt="dcsc", form="numeric_reuse", reps=1,
                      space=AT.REPLAY_SPACE, presets=AT.REPLAY_PRESETS)
    # the default, every preset (none refused) and at least one space value were timed
    assert res["tried"] >= 2 + len(AT.REPLAY_PRESETS)
    plan = BT.summa_share_plan(semiring, dA, dB, tuning=sg.make_tuning(semiring, **res["tuning"]))
    G = BT.GraphedNumeric(plan)
    G.replay()
    G.replay()
    assert_same(G.outputs[0].to_host(), R, semiring, 1e-12, f"tuned replay {res['tuning']}")
    plan.destroy()


@pytest.mark.parametrize("force", [-1, 1, 2, 3])
def test_summa_share_many_segments(sg, force):
    """16 stage products per output vector (more segments than wavefronts per workgroup), every tier."""
    from paper_1006_2183_amd import batched as BT
    semiring = "plus_times_f64"
    scale, grid = 12, 16
    _say(f"case summa share 16 stages force {force}")
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (3, 5), semiring=semiring, seed=17)
    b = (1 << scale) // grid
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in b_blocks]
    SA, SB = strips(a_blocks, b_blocks, b, grid, semiring)
    R, _ = oracle.spgemm(semiring, SA, SB)
    for batched in (False, True):
        t = sg.make_tuning(semiring, force_tier=force, lds_bytes=24576, block_threads=512, heavy_lds_bytes=24576,
                           heavy_threads=512)
        C = BT.summa_share(semiring, dA, dB, tuning=t, batched=batched).to_host()
        assert_canonical(C)
        assert_same(C, R, semiring, 1e-12, f"force {force} batched {batched}")


@pytest.mark.parametrize("semiring", ["plus_times_f64", "min_plus_i32"])
@pytest.mark.parametrize("entry_mb", [1, 2048])
@pytest.mark.parametrize("force", [2, -1, 3])
def test_summa_share_entry_records(sg, semiring, entry_mb, force):
    """Heavy windows (and, unforced, mid-tier vectors) fed by 16 stage products, walked from
    entry records (all, or some within a 1 MiB budget), per tier launch and in the
    persistent launch."""
    from paper_1006_2183_amd import batched as BT
    scale, grid = 16, 16  # blocks of 4096 ids: wider than one dense window, so rank windows and records
    _say(f"case summa share entry records {semiring} entry_mb={entry_mb} force {force}")
    a_blocks, b_blocks = W.summa_share(scale, 16, grid, (3, 5), semiring=semiring, seed=17)
    b = (1 << scale) // grid
    dA = [sg.DevMat.from_host(x, "cuda", semiring) for x in a_blocks]
    dB = [sg.DevMat.from_host(x, "cuda", semiring) for x in b_blocks]
    SA, SB = strips(a_blocks, b_blocks, b, grid, semiring)
    R, _ = oracle.spgemm(semiring, SA, SB)
    for batched in (False, True):
        t = sg.make_tuning(semiring, force_tier=force, lds_bytes=24576, block_threads=512, heavy_lds_bytes=24576,
                           heavy_threads=512, entry_mb=entry_mb)
        C = BT.summa_share(semiring, dA, dB, tuning=t, batched=batched).to_host()
        assert_canonical(C)
        assert_same(C, R, semiring, 1e-12, f"entry_mb {entry_mb} batched {batched} force {force}")
