"""Method-level work count of the peeling method (TEST INFRASTRUCTURE ONLY, like
the rest of this package): how many edge-support evaluations, and how many
bytes, the re-evaluating form of Algorithm 1 (Section 3) needs on a given
graph, counted from the definitions on the bulk round schedule.

Notation: S_r is the edge set before round r (S_0 = E), R_r the edges round r
removes, B_S(x, j) = {y : dist_S(x, y) <= j} (x included) and
N_S(x, j) = B_S(x, j) minus x (Section 2).

  Evaluations  E_eval = m + sum_r |A_r|: every edge once at the start, then in
               round r the edges of S_{r+1} with an endpoint whose h-ball
               changed, D(x) = N_{S_r}(x, h) minus N_{S_{r+1}}(x, h) non-empty
               (h-support depends only on the two endpoint balls, Def. 3).
  Bytes        B_alg = sum over evaluations e = (u, v) in S of s(u) + s(v) + 4,
                       s(x) = min(4 |N_S(x, h)|, ceil(n / 8))  (the smaller exact
                       encoding of a ball: a u32 list or a bitset),
               + sum over ball builds of
                       b(x) = min(sum over y in B_S(x, h-1) of 8 + 4 deg_S(y),
                                  h (4 (n+1) + 8 |S| + ceil(n / 8)))
                       (frontier reads of a bounded BFS, or h full scans),
               ball builds: every non-isolated vertex of G at the start, then
               in round r every x in V_cand = the union of B_{S_r}(z, h-1) over
               the endpoints z of R_r, built in S_{r+1}.
Rounds after which nothing is left (S_{r+1} empty) evaluate and build
nothing.  Reachability is computed with dense boolean matrix products, so
this is for small graphs (n up to a few thousand).
"""
from __future__ import annotations

import numpy as np


def _reach(n: int, eu: np.ndarray, ev: np.ndarray, keep: np.ndarray, hops: int) -> np.ndarray:
    """reach[x, y] = dist_S(x, y) <= hops, S = the edges with keep set."""
    A = np.zeros((n, n), dtype=np.float32)
    A[eu[keep], ev[keep]] = 1.0
    A[ev[keep], eu[keep]] = 1.0
    R = np.eye(n, dtype=bool)
    for _ in range(hops):
        R = R | ((R.astype(np.float32) @ A) > 0)
    return R


def _edges(g):
    """Endpoints (u < v) of every edge in canonical order."""
    rp = g.row_ptr.astype(np.int64)
    ci = g.col_idx.astype(np.int64)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    up = ci > src
    return src[up], ci[up]


def count(g, h: int, rho: np.ndarray, keep_sets: bool = False) -> dict:
    """E_eval, B_alg and |A_r| per round for the bulk schedule rho (the round
    in which each edge is removed, as the peeling oracle returns it); with
    keep_sets, also the edge ids of every A_r."""
    n = g.n
    eu, ev = _edges(g)
    m = eu.size
    cap = h * (4 * (n + 1)) + h * ((n + 7) // 8)  # plus h * 8|S|, added per S
    nb = (n + 7) // 8

    def s_of(ball_rows):
        return np.minimum(4 * (ball_rows.sum(axis=1) - 1), nb)

    def builds(keep, xs):
        deg = np.zeros(n, dtype=np.int64)
        np.add.at(deg, eu[keep], 1)
        np.add.at(deg, ev[keep], 1)
        Rb = _reach(n, eu, ev, keep, h - 1)
        frontier = (Rb[xs].astype(np.int64) * (8 + 4 * deg)[None, :]).sum(axis=1)
        return int(np.minimum(frontier, cap + 8 * h * int(keep.sum())).sum())

    everything = np.ones(m, dtype=bool)
    B0 = _reach(n, eu, ev, everything, h)
    s0 = s_of(B0)
    evals = m
    nbytes = int((s0[eu] + s0[ev] + 4).sum())
    deg0 = np.zeros(n, dtype=np.int64)
    np.add.at(deg0, eu, 1)
    np.add.at(deg0, ev, 1)
    nbytes += builds(everything, np.nonzero(deg0 > 0)[0])
    rounds = int(rho.max()) + 1 if m else 0
    per_round = []
    sets = []
    Bold = B0
    for r in range(rounds):
        keep_now = rho >= r
        keep_next = rho >= r + 1
        Bnew = _reach(n, eu, ev, keep_next, h)
        if not keep_next.any():
            per_round.append(0)
            break
        changed = (Bold != Bnew).any(axis=1)
        A = keep_next & (changed[eu] | changed[ev])
        sn = s_of(Bnew)
        per_round.append(int(A.sum()))
        if keep_sets:
            sets.append(np.nonzero(A)[0])
        evals += int(A.sum())
        nbytes += int((sn[eu[A]] + sn[ev[A]] + 4).sum())
        removed = rho == r
        Rold = _reach(n, eu, ev, keep_now, h - 1)
        ends = np.unique(np.concatenate([eu[removed], ev[removed]]))
        vcand = np.nonzero(Rold[ends].any(axis=0))[0]
        nbytes += builds(keep_next, vcand)
        Bold = Bnew
    out = {"evaluations": evals, "alg_bytes": nbytes, "a_sizes": np.array(per_round)}
    if keep_sets:
        out["a_sets"] = sets
    return out
