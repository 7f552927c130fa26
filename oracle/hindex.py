"""The H-index fixpoint method of Section 4, the plain way (TEST INFRASTRUCTURE
ONLY, like the rest of this package).

Section 4.1 defines, for edge keys H(e) >= 0:
  * the H-index operator: H(S) is the largest y such that at least y members
    of the multiset S are >= y (0 for an empty S);
  * the h-hop reachable path key P(x, w): the largest, over paths from x to w
    with at most h edges, of the smallest key on the path (the paper's
    "distance <= h" is read as "path length <= h");
  * the higher-order H-index sequence: H^(0)(e) = sup_G(e, h) (Def. 3) and
    H^(n)(u, v) = H({min(P(u, w), P(v, w)) : w in the common h-hop
    neighbourhood of u and v in G}), with P taken over the keys H^(n-1).
Theorem 1 makes the sequence non-increasing and Theorem 2 makes it reach
t(e, h) - 2.  The synchronous iteration (Algorithm 2) recomputes every edge
from the previous sweep's keys and stops at the first sweep that changes
nothing; that sweep is counted.

Path keys are computed by h rounds of relaxation over walks (a walk of at most
h edges contains a path of at most h edges whose smallest key is no smaller,
so the maximum over walks equals the maximum over paths).  The common
neighbourhood uses hop distances in G, which the same relaxation yields: w is
within h hops of x exactly when some walk of at most h edges reaches it.
"""
from __future__ import annotations

import numpy as np

from .oracle import h_support

UNREACHED = -1


def hindex(values) -> int:
    """H(S): the largest y with at least y members of S no smaller than y."""
    s = np.sort(np.asarray(values, dtype=np.int64))[::-1]
    y = 0
    while y < s.size and s[y] >= y + 1:
        y += 1
    return y


def path_keys(n: int, ends: np.ndarray, key: np.ndarray, h: int, src: int) -> np.ndarray:
    """P(src, w) for every vertex w (UNREACHED beyond h hops; P(src, src) is
    left UNREACHED, it is never used).  ends: (m, 2) edge endpoints, key: (m,)."""
    big = np.iinfo(np.int64).max
    a = np.concatenate([ends[:, 0], ends[:, 1]]).astype(np.int64)
    b = np.concatenate([ends[:, 1], ends[:, 0]]).astype(np.int64)
    k = np.concatenate([key, key]).astype(np.int64)
    p = np.full(n, UNREACHED, dtype=np.int64)
    p[src] = big                                  # the empty walk
    for _ in range(h):
        q = p.copy()                              # walks of one more edge
        ok = p[a] != UNREACHED
        np.maximum.at(q, b[ok], np.minimum(p[a[ok]], k[ok]))
        p = q
    p[src] = UNREACHED
    return p


def sweep(g, h: int, H: np.ndarray) -> np.ndarray:
    """One synchronous update: H^(n) from H^(n-1)."""
    ends = g.edges().astype(np.int64)
    P = np.stack([path_keys(g.n, ends, H, h, x) for x in range(g.n)]) if g.n else None
    out = np.empty_like(H)
    for i, (u, v) in enumerate(ends):
        pu, pv = P[u], P[v]
        common = (pu != UNREACHED) & (pv != UNREACHED)
        common[u] = common[v] = False
        out[i] = hindex(np.minimum(pu[common], pv[common]))
    return out


def hindex_sequence(g, h: int, max_sweeps: int = 0) -> list:
    """[H^(0), H^(1), ..., H^(N)]: the synchronous iteration up to and
    including the first sweep N that changes nothing (or N = max_sweeps when
    that is positive and reached first).  N is the sweep count."""
    H = h_support(g, h).astype(np.int64)
    seq = [H]
    if g.m == 0:
        return seq
    while True:
        nxt = sweep(g, h, seq[-1])
        seq.append(nxt)
        if np.array_equal(nxt, seq[-2]) or (max_sweeps and len(seq) - 1 >= max_sweeps):
            return seq


def hindex_trussness(g, h: int):
    """(t = H^(N) + 2 per edge, sweep count N) of the synchronous iteration."""
    seq = hindex_sequence(g, h)
    return (seq[-1] + 2).astype(np.uint32), len(seq) - 1
