"""CPU oracle of the masked multi-level breadth-first search (test
infrastructure only; the same import rules as the rest of ``oracle``).

Multi-source BFS as repeated sparse products (paper, Section 6.2.2): with A
the n x n adjacency matrix in column-major form (A(i, k) stored: an edge from
k to i) and X_0 the n x k frontier holding source s_c in column c, level d+1
is X_{d+1} = (A X_d) with the positions already visited removed, and the
visited set grows by X_{d+1}. Here each column is its own search, so
"visited" is per column.

Plain Python sets, one search per column: frontier, then for each frontier
vertex u every i with A(i, u) stored, minus the visited set. Returns, per
column, the list of level sets (level 0 is the source).
"""
from __future__ import annotations

import numpy as np


def bfs_levels(A, sources, max_levels=None):
    """levels[c][d] = sorted int array of the vertices first reached at depth d
    from sources[c] (levels[c][0] = [sources[c]])."""
    ptr = np.asarray(A.ptr, dtype=np.int64)
    idx = np.asarray(A.idx, dtype=np.int64)
    if A.fmt != "csc":
        raise ValueError("column-major adjacency expected (csc)")
    out = []
    for s in sources:
        s = int(s)
        seen = {s}
        front = [s]
        levels = [np.array([s], dtype=np.int64)]
        while front and (max_levels is None or len(levels) < max_levels + 1):
            nxt = set()
            for u in front:
                for i in idx[ptr[u]:ptr[u + 1]]:
                    i = int(i)
                    if i not in seen:
                        nxt.add(i)
            if not nxt:
                break
            seen |= nxt
            front = sorted(nxt)
            levels.append(np.array(front, dtype=np.int64))
        out.append(levels)
    return out


def level_matrix(levels, d, n):
    """Frontier of depth d as (rows, cols): the vertices of column c at depth d."""
    rows, cols = [], []
    for c, lv in enumerate(levels):
        if d < len(lv):
            rows.append(lv[d])
            cols.append(np.full(lv[d].size, c, dtype=np.int64))
    if not rows:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(rows), np.concatenate(cols)
