"""Brute-force h-trussness straight from the definitions, for tiny graphs.

TEST INFRASTRUCTURE ONLY.  Independent of peeling: for every edge subset S it
evaluates min over f in S of sup_S(f,h) and gives each e in S the value
min + 2 if that beats what e already has.  By Def. 4 (Section 2) the
h-trussness of e is the largest k for which some S containing e has
sup_S(f,h) >= k-2 on all its edges, which is exactly that maximum.
Cost is 2^m subsets, so keep m at about 14 or below.
"""
from __future__ import annotations

import numpy as np


def _closed_balls(nv: int, adj: list, h: int) -> list:
    """ball[x] = bitmask of vertices at distance <= h from x using adj (x included)."""
    ball = [1 << x for x in range(nv)]
    for _ in range(h):
        nxt = []
        for x in range(nv):
            b = ball[x]
            acc = b
            while b:
                low = b & -b
                acc |= adj[low.bit_length() - 1]
                b ^= low
            nxt.append(acc)
        ball = nxt
    return ball


def _sup_in_subset(nv, edges, mask, h):
    """sup_S(f,h) for f in S = {edges[i] : bit i of mask}; Def. 3 with N(x,h)
    excluding x, so neither endpoint is ever a common h-neighbour."""
    adj = [0] * nv
    idx = []
    i = 0
    mm = mask
    while mm:
        if mm & 1:
            u, v = edges[i]
            adj[u] |= 1 << v
            adj[v] |= 1 << u
            idx.append(i)
        mm >>= 1
        i += 1
    ball = _closed_balls(nv, adj, h)
    out = {}
    for i in idx:
        u, v = edges[i]
        common = ball[u] & ball[v] & ~(1 << u) & ~(1 << v)
        out[i] = bin(common).count("1")
    return out


def brute_h_support(g, h: int, live=None) -> np.ndarray:
    """sup_S(e,h) for every edge of g; S = edges with live[e] true (all if None)."""
    edges = [tuple(map(int, e)) for e in g.edges()]
    m = len(edges)
    mask = 0
    for i in range(m):
        if live is None or live[i]:
            mask |= 1 << i
    sup = _sup_in_subset(g.n, edges, mask, h)
    return np.array([sup.get(i, 0) for i in range(m)], dtype=np.uint32)


def brute_trussness(g, h: int) -> np.ndarray:
    """t(e,h) = max over S containing e of (min_{f in S} sup_S(f,h) + 2)."""
    edges = [tuple(map(int, e)) for e in g.edges()]
    m = len(edges)
    if m > 20:
        raise ValueError("brute force limited to m <= 20")
    best = [2] * m
    for mask in range(1, 1 << m):
        sup = _sup_in_subset(g.n, edges, mask, h)
        val = min(sup.values()) + 2
        for i in sup:
            if val > best[i]:
                best[i] = val
    return np.array(best, dtype=np.uint32)
