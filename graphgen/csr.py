"""Undirected simple graphs in CSR form (input preparation only).

A graph is stored the way the library's boundary takes it: ``row_ptr``
(uint32, n+1 entries) and ``col_idx`` (uint32, 2m entries), symmetric (both
directions of every edge present), each row sorted ascending, no self-loops and
no duplicate entries.  Isolated vertices are allowed.

The canonical undirected edge order is the upper-triangle CSR order: for
x = 0..n-1 ascending, every neighbour y > x of x ascending.  The rank of
(x, y) in that order is its edge id; the per-edge outputs of both the oracle
and the GPU path are laid out in it.  This module holds no part of the truss
computation itself.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # uint32 [n+1]
    col_idx: np.ndarray  # uint32 [2m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1]) // 2

    def edges(self) -> np.ndarray:
        """Canonical (m, 2) uint32 array of (u, v) with u < v, in edge-id order."""
        deg = np.diff(self.row_ptr.astype(np.int64))
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.col_idx.astype(np.int64)
        keep = dst > src
        return np.stack([src[keep], dst[keep]], axis=1).astype(np.uint32)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def summary(self) -> dict:
        deg = self.degrees()
        return {
            "name": self.name,
            "n": int(self.n),
            "m": int(self.m),
            "isolated": int((deg == 0).sum()),
            "max_deg": int(deg.max()) if self.n else 0,
            "sum_deg_sq": int((deg * deg).sum()),
            **self.meta,
        }


def from_edges(n: int, u, v, name: str = "", meta: dict | None = None) -> Graph:
    """Build a simple undirected CSR graph from endpoint arrays.

    Self-loops are dropped, each pair is canonicalised to (min, max) and
    duplicates are removed; both directions are then stored.
    """
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.shape != v.shape:
        raise ValueError("endpoint arrays differ in length")
    if n < 0 or n >= 2**32 - 1:
        raise ValueError("n out of range for uint32 ids")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("endpoint outside [0, n)")
    keep = u != v
    a = np.minimum(u[keep], v[keep])
    b = np.maximum(u[keep], v[keep])
    key = np.unique(a * np.int64(n) + b)
    a = key // n
    b = key % n
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    if src.size >= 2**32:
        raise ValueError("too many adjacency entries for uint32 CSR")
    counts = np.bincount(src, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=int(n), row_ptr=row_ptr.astype(np.uint32),
                 col_idx=dst.astype(np.uint32), name=name, meta=dict(meta or {}))


def from_edge_list(n: int, edges, name: str = "", meta: dict | None = None) -> Graph:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return from_edges(n, e[:, 0], e[:, 1], name=name, meta=meta)


def validate(g: Graph) -> None:
    """Raise ValueError unless g is a symmetric, sorted, loop-free simple CSR."""
    rp = g.row_ptr.astype(np.int64)
    ci = g.col_idx.astype(np.int64)
    if rp.shape != (g.n + 1,) or rp[0] != 0 or np.any(np.diff(rp) < 0):
        raise ValueError("row_ptr malformed")
    if rp[-1] != ci.size or ci.size % 2:
        raise ValueError("row_ptr[n] must equal len(col_idx), which must be even")
    if ci.size and (ci.min() < 0 or ci.max() >= g.n):
        raise ValueError("col_idx out of range")
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rp))
    if np.any(src == ci):
        raise ValueError("self-loop")
    same_row = src[1:] == src[:-1]
    if np.any(same_row & (ci[1:] <= ci[:-1])):
        raise ValueError("row not strictly ascending (duplicate or unsorted)")
    fwd = np.sort(src * g.n + ci)
    bwd = np.sort(ci * g.n + src)
    if not np.array_equal(fwd, bwd):
        raise ValueError("adjacency not symmetric")


def disjoint_union(graphs) -> Graph:
    """Vertex-disjoint union; graph i's vertices are shifted by sum of earlier n."""
    us, vs = [], []
    off = 0
    for g in graphs:
        e = g.edges().astype(np.int64)
        us.append(e[:, 0] + off)
        vs.append(e[:, 1] + off)
        off += g.n
    if not us:
        return from_edges(0, [], [])
    return from_edges(off, np.concatenate(us), np.concatenate(vs), name="union")


@dataclass
class Batch:
    """Many graphs concatenated for a single batched call.

    row_ptr_cat holds each graph's local (n_g+1)-entry row_ptr back to back, so
    graph g's segment starts at index vtx_off[g] + g; col_idx_cat holds local
    vertex ids, graph g's segment starting at adj_off[g]; per-edge outputs of
    graph g start at edge_off[g].
    """
    graphs: list
    h: np.ndarray         # uint32 [B]
    row_ptr_cat: np.ndarray
    col_idx_cat: np.ndarray
    vtx_off: np.ndarray   # uint64 [B+1]
    adj_off: np.ndarray   # uint64 [B+1]
    edge_off: np.ndarray  # uint64 [B+1]

    @property
    def B(self) -> int:
        return len(self.graphs)


def concat(graphs, h) -> Batch:
    h = np.broadcast_to(np.asarray(h, dtype=np.uint32), (len(graphs),)).copy()
    n = np.array([g.n for g in graphs], dtype=np.uint64)
    a = np.array([g.col_idx.size for g in graphs], dtype=np.uint64)
    vtx_off = np.zeros(len(graphs) + 1, dtype=np.uint64)
    adj_off = np.zeros(len(graphs) + 1, dtype=np.uint64)
    np.cumsum(n, out=vtx_off[1:])
    np.cumsum(a, out=adj_off[1:])
    edge_off = adj_off // 2
    rp = np.concatenate([g.row_ptr for g in graphs]) if graphs else np.zeros(0, np.uint32)
    ci = np.concatenate([g.col_idx for g in graphs]) if graphs else np.zeros(0, np.uint32)
    return Batch(list(graphs), h, rp.astype(np.uint32), ci.astype(np.uint32),
                 vtx_off, adj_off, edge_off)
