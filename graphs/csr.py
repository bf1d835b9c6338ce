"""CSR packing of simple undirected graphs.

A graph is finite, simple and undirected (paper §II-A). It is stored as int32 CSR:
``row_ptr[n+1]`` and ``col_idx[nnz]`` with ``nnz = 2|E|``; every edge appears in both
rows, each row is sorted ascending, there are no self-loops and no duplicates.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class CSRGraph:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz]
    meta: dict = field(default_factory=dict, compare=False)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int32)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]


def from_edges(n: int, u, v, meta: dict | None = None) -> CSRGraph:
    """Pack an undirected edge list into sorted symmetric int32 CSR.

    Raises ``ValueError`` on a self-loop, a duplicate edge or an id outside [0, n).
    """
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.shape != v.shape:
        raise ValueError("edge endpoint arrays differ in length")
    if n < 0:
        raise ValueError("negative vertex count")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("edge endpoint out of range")
    if np.any(u == v):
        raise ValueError("self-loop")
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = lo * max(n, 1) + hi
    if np.unique(key).size != key.size:
        raise ValueError("duplicate edge")
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return CSRGraph(n, row_ptr.astype(np.int32), dst.astype(np.int32), dict(meta or {}))


def edges_of(g: CSRGraph) -> tuple[np.ndarray, np.ndarray]:
    """Each undirected edge once, as (u, v) with u < v."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col_idx.astype(np.int64)
    keep = src < dst
    return src[keep], dst[keep]


def disjoint_union(*gs: CSRGraph) -> CSRGraph:
    us, vs = [], []
    off = 0
    for g in gs:
        u, v = edges_of(g)
        us.append(u + off)
        vs.append(v + off)
        off += g.n
    if not us:
        return from_edges(0, [], [])
    return from_edges(off, np.concatenate(us), np.concatenate(vs))
