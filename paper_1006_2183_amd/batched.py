"""Batched forms of the local product: one plan for many products.

* ``summa_share``: the local work of one Sparse SUMMA process, C_IJ =
  (+)_k A_Ik (x) A_kJ over all stages k (paper, Sections 3.2 and 3.5). All
  stage products form one group, so the stage partials are accumulated in
  the same output vectors instead of being materialised and merged.
* ``merge_partials``: the materialise-then-merge alternative: the stage
  partials C_k are summed by a grouped product with an identity operand
  (C = (+)_k I C_k column-major), a k-way merge on the same accumulators.
* ``galerkin_rap``: R (A P) for many uneven instances (graph contraction and
  multigrid coarsening, Section 6.2.3), two grouped plans (A P, then R (AP)).
* ``galerkin_fused``: the same triple products as one fused chain plan: the
  intermediate A P is never written to memory.
* ``GraphedNumeric``: captures the persistent batched launches of one plan
  or a chain of plans in a HIP graph; each replay recomputes the outputs
  from the current operand values (same structure), with no host work.

All arithmetic runs in the HIP library; this module arranges plans and
PyTorch-owned buffers.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

from . import binding as B
from .binding import DevMat


def summa_share(semiring: str, A_blocks: Sequence[DevMat], B_blocks: Sequence[DevMat], out_fmt: str = "dcsc",
                tuning=None, batched: bool = True, stream=None) -> DevMat:
    """C_IJ = (+)_k A_blocks[k] (x) B_blocks[k], every stage product in one plan."""
    n = len(A_blocks)
    Cs = B.spgemm_grouped(semiring, list(A_blocks), list(B_blocks), [0] * n, 1, out_fmt=out_fmt, tuning=tuning,
                          batched=batched, stream=stream)
    return Cs[0]


def summa_share_plan(semiring: str, A_blocks, B_blocks, out_fmt: str = "dcsc", tuning=None, stream=None):
    """The plan of ``summa_share`` (symbolic phase only), for repeated numeric phases.

    A plan that is replayed many times gains from per-window entry records
    (``entry_mb`` in the tuning): its symbolic phase writes them once and
    every numeric phase reads one record per streamed entry instead of
    walking the 64 stage products' descriptors.
    """
    n = len(A_blocks)
    return B.spgemm_symbolic(semiring, list(A_blocks), list(B_blocks), [0] * n, 1, out_fmt=out_fmt,
                             tuning=tuning, stream=stream)


def identity(n: int, semiring: str, fmt: str, device) -> DevMat:
    """n x n identity with the semiring's multiplicative unit (as a device matrix)."""
    import torch
    one = {"plus_times_f64": (torch.float64, 1.0), "plus_times_f32": (torch.float32, 1.0),
           "min_plus_i32": (torch.int32, 0), "or_and_bool": (None, None)}[semiring]
    ptr = torch.arange(n + 1, dtype=torch.int64, device=device)
    idx = torch.arange(n, dtype=torch.int32, device=device)
    val = None if one[0] is None else torch.full((n,), one[1], dtype=one[0], device=device)
    vid = torch.arange(n, dtype=torch.int32, device=device) if fmt in ("dcsr", "dcsc") else None
    return DevMat(fmt, n, n, ptr, idx, val, vid)


def merge_partials(semiring: str, partials: Sequence[DevMat], out_fmt: Optional[str] = None, tuning=None,
                   batched: bool = True, stream=None) -> DevMat:
    """(+)_k partials[k] as one grouped product with identity operands (a k-way merge)."""
    C0 = partials[0]
    col = C0.fmt in ("csc", "dcsc")
    dev = C0.ptr.device
    fmt = C0.fmt
    # the partials are the streamed operand, so the output vectors are only
    # their stored vectors: I C_k column-major, C_k I row-major
    if col:
        I = identity(C0.nrows, semiring, "csc", dev)
        As, Bs = [I] * len(partials), list(partials)
    else:
        I = identity(C0.ncols, semiring, "csr", dev)
        As, Bs = list(partials), [I] * len(partials)
    Cs = B.spgemm_grouped(semiring, As, Bs, [0] * len(partials), 1, out_fmt=out_fmt or fmt, tuning=tuning,
                          batched=batched, stream=stream)
    return Cs[0]


def galerkin_rap(semiring: str, Rs: Sequence[DevMat], As: Sequence[DevMat], Ps: Sequence[DevMat], tuning=None,
                 batched: bool = True, stream=None) -> List[DevMat]:
    """R_i (A_i P_i) for every instance i: two grouped plans, one output per instance."""
    n = len(As)
    AP = B.spgemm_grouped(semiring, list(As), list(Ps), list(range(n)), n, tuning=tuning, batched=batched,
                          stream=stream)
    return B.spgemm_grouped(semiring, list(Rs), AP, list(range(n)), n, tuning=tuning, batched=batched,
                            stream=stream)


def galerkin_plans(semiring: str, Rs: Sequence[DevMat], As: Sequence[DevMat], Ps: Sequence[DevMat], tuning=None,
                   stream=None):
    """Plans of the two grouped products of ``galerkin_rap`` for repeated numeric phases.

    Returns (plan_ap, ap_outputs, plan_rap): the second plan reads the first
    plan's outputs, so running the two persistent launches in order (or
    replaying them in one graph) recomputes R (A P) from the current values.
    """
    n = len(As)
    plan_ap = B.spgemm_symbolic(semiring, list(As), list(Ps), list(range(n)), n, tuning=tuning, stream=stream)
    AP = plan_ap.alloc_outputs(As[0].ptr.device)
    B.spgemm_batched(plan_ap, AP, stream)
    plan_rap = B.spgemm_symbolic(semiring, list(Rs), AP, list(range(n)), n, tuning=tuning, stream=stream)
    return plan_ap, AP, plan_rap


def galerkin_chain_plan(semiring: str, Rs: Sequence[DevMat], As: Sequence[DevMat], Ps: Sequence[DevMat], tuning=None,
                        stream=None):
    """One fused plan for every instance's R_i A_i P_i: the products A P are never
    written; the plan's numeric phase (plain, batched or graph-replayed) recomputes
    every R A P from the current values of R, A and P, so a repeated setup with new
    values reuses this symbolic phase."""
    return B.chain_symbolic(semiring, list(Rs), list(As), list(Ps), tuning=tuning, stream=stream)


def galerkin_fused(semiring: str, Rs: Sequence[DevMat], As: Sequence[DevMat], Ps: Sequence[DevMat], tuning=None,
                   batched: bool = True, stream=None) -> List[DevMat]:
    """R_i A_i P_i for every instance, fused (one plan, one output per instance)."""
    plan = galerkin_chain_plan(semiring, Rs, As, Ps, tuning=tuning, stream=stream)
    C = plan.alloc_outputs(As[0].ptr.device)
    (B.spgemm_batched if batched else B.spgemm_numeric)(plan, C, stream)
    plan.destroy()
    return C


class GraphedNumeric:
    """The persistent batched launches of one or more plans captured in one HIP graph
    (torch.cuda.CUDAGraph), in order.

    The outputs are allocated once (or passed in: a later plan may read an
    earlier plan's outputs, as R (A P) reads A P); ``replay()`` recomputes
    them from the current values of the operands the plans were built on.
    """

    def __init__(self, plans, outputs: Optional[List[List[DevMat]]] = None):
        import torch
        self.plans = list(plans) if isinstance(plans, (list, tuple)) else [plans]
        if outputs is None:
            outputs = [None] * len(self.plans)
        elif isinstance(outputs[0], DevMat):
            outputs = [outputs]
        self.outs = [o if o is not None else p.alloc_outputs(p.As[0].ptr.device) for p, o in zip(self.plans, outputs)]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for p, o in zip(self.plans, self.outs):
                B.spgemm_batched(p, o, side)  # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for p, o in zip(self.plans, self.outs):
                B.spgemm_batched(p, o, torch.cuda.current_stream())

    @property
    def outputs(self) -> List[DevMat]:
        return self.outs[-1]

    def replay(self) -> List[DevMat]:
        """Replays the graph; returns the last plan's outputs."""
        self.graph.replay()
        return self.outs[-1]
