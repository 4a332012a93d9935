"""Seeded synthetic inputs for the local SpGEMM C = A (x) B.

This module builds operands only. It holds none of the product's arithmetic:
no semiring multiply, no accumulation across a shared dimension. Both the
CPU oracle and the GPU library consume the matrices made here, and neither
imports the other.

Workloads follow the paper's synthetic families (Section 5.1 and 6.2):

* R-MAT scale-free adjacency matrices (Section 5.1.1), with the quadrant
  probabilities passed in (the survey fixes 0.57/0.19/0.19/0.05),
* the 3D 7-point grid (Section 5.1.3) and a 2x2x2 aggregation
  restriction/prolongation pair, as in graph contraction (Section 6.2.3),
* the 2D block share of one Sparse SUMMA process after a random symmetric
  relabelling (Sections 3.2, 3.5 and 7.1),
* multi-source BFS frontiers for tall-skinny right-hand sides (Section 6.2.2).

Duplicate coordinates in a generated triple list are combined with the
semiring's add (sum, min or logical or) while the canonical compressed form
is built; this is input construction, not the product.
"""
from .matrices import SpMat, from_triples, to_format, random_values, VALUE_DTYPES
from .gen import (
    rmat_edges,
    rmat_matrix,
    laplacian_7pt,
    aggregation_p,
    transpose,
    summa_share,
    bfs_frontier,
    poisson_arrivals,
    random_sparse,
    permutation_matrix,
    identity_matrix,
)

__all__ = [
    "SpMat", "from_triples", "to_format", "random_values", "VALUE_DTYPES",
    "rmat_edges", "rmat_matrix", "laplacian_7pt", "aggregation_p", "transpose",
    "summa_share", "bfs_frontier", "poisson_arrivals", "random_sparse",
    "permutation_matrix", "identity_matrix",
]
