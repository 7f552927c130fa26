"""Seeded synthetic graph generators (input preparation only).

These stand in for the public network datasets the paper measures on, which
are not available here; each generator reproduces the shape of one workload
class (uniform random, power-law Chung-Lu, R-MAT, preferential attachment with
planted cliques) plus the small closed-form families used as pins.  Every
generator is deterministic in its seed (numpy PCG64).  Nothing here computes
any part of the truss decomposition.
"""
from __future__ import annotations

import numpy as np

from .csr import Graph, from_edges


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# closed-form families
# --------------------------------------------------------------------------

def complete(n: int) -> Graph:
    iu, iv = np.triu_indices(n, 1)
    return from_edges(n, iu, iv, name=f"K{n}")


def cycle(n: int) -> Graph:
    if n < 3:
        raise ValueError("cycle needs n >= 3")
    a = np.arange(n)
    return from_edges(n, a, (a + 1) % n, name=f"C{n}")


def path(num_edges: int) -> Graph:
    a = np.arange(num_edges)
    return from_edges(num_edges + 1, a, a + 1, name=f"P{num_edges}")


def star(r: int) -> Graph:
    return from_edges(r + 1, np.zeros(r, np.int64), np.arange(1, r + 1), name=f"S{r}")


def empty(n: int) -> Graph:
    return from_edges(n, [], [], name=f"E{n}")


# --------------------------------------------------------------------------
# random families
# --------------------------------------------------------------------------

def erdos_renyi(n: int, p: float, seed=0) -> Graph:
    """G(n, p): every pair u < v kept independently with probability p."""
    rng = _rng(seed)
    iu, iv = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    return from_edges(n, iu[keep], iv[keep], name=f"ER({n},{p})",
                      meta={"seed": seed, "gen": "er"})


def random_small(n: int, max_edges: int, seed=0) -> Graph:
    """A uniformly chosen set of at most max_edges distinct pairs on n vertices."""
    rng = _rng(seed)
    iu, iv = np.triu_indices(n, 1)
    k = int(rng.integers(0, min(max_edges, iu.size) + 1))
    pick = rng.choice(iu.size, size=k, replace=False)
    return from_edges(n, iu[pick], iv[pick], name=f"rand({n},{k})",
                      meta={"seed": seed, "gen": "random_small"})


def chung_lu(n: int, avg_deg: float, gamma: float, seed=0) -> Graph:
    """Chung-Lu power-law graph.

    Weights w_i proportional to (i+1)^(-1/(gamma-1)), scaled to mean avg_deg;
    n*avg_deg/2 endpoint pairs are drawn independently with P(i) ~ w_i;
    self-loops and repeated pairs are dropped.
    """
    rng = _rng(seed)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= avg_deg / w.mean()
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    M = int(round(n * avg_deg / 2.0))
    u = np.searchsorted(cdf, rng.random(M), side="right")
    v = np.searchsorted(cdf, rng.random(M), side="right")
    u = np.minimum(u, n - 1)
    v = np.minimum(v, n - 1)
    return from_edges(n, u, v, name=f"ChungLu({n},{avg_deg},{gamma})",
                      meta={"seed": seed, "gen": "chung_lu", "gamma": gamma,
                            "avg_deg": avg_deg})


def rmat(scale: int, edge_factor: int = 16, abcd=(0.57, 0.19, 0.19, 0.05),
         seed=0) -> Graph:
    """R-MAT: edge_factor * 2^scale endpoint pairs by recursive quadrant choice,
    then a seeded vertex permutation, symmetrised, loops and duplicates dropped."""
    rng = _rng(seed)
    n = 1 << scale
    E = edge_factor * n
    a, b, c, d = abcd
    u = np.zeros(E, dtype=np.int64)
    v = np.zeros(E, dtype=np.int64)
    t1, t2, t3 = a, a + b, a + b + c
    for _ in range(scale):
        r = rng.random(E)
        bu = (r >= t2).astype(np.int64)                      # quadrants c, d
        bv = (((r >= t1) & (r < t2)) | (r >= t3)).astype(np.int64)  # b, d
        u = (u << 1) | bu
        v = (v << 1) | bv
    perm = rng.permutation(n)
    return from_edges(n, perm[u], perm[v], name=f"RMAT{scale}",
                      meta={"seed": seed, "gen": "rmat", "scale": scale,
                            "edge_factor": edge_factor})


def barabasi_albert(n: int, m_attach: int, seed=0, rng=None):
    """Preferential attachment: start from a clique on m_attach+1 vertices; each
    later vertex draws m_attach targets from the repeated-endpoint list as it
    stood before that vertex arrived (repeats merged).  Returns endpoint arrays.

    The draws are resolved without a per-vertex Python loop: every target slot
    points to an earlier list position; positions holding earlier targets are
    followed (pointer jumping) until they land on a source entry.
    """
    rng = rng if rng is not None else _rng(seed)
    m0 = m_attach + 1
    if n <= m0:
        iu, iv = np.triu_indices(n, 1)
        return iu.astype(np.int64), iv.astype(np.int64)
    iu, iv = np.triu_indices(m0, 1)
    init = np.concatenate([iu, iv]).astype(np.int64)      # endpoint list of the seed clique
    L0 = init.size
    newv = np.arange(m0, n, dtype=np.int64)
    k = newv.size
    blk = 2 * m_attach
    start = L0 + (newv - m0) * blk                         # list length before vertex arrives
    # list layout after the seed: per new vertex, m sources then m targets
    total = L0 + k * blk
    val = np.full(total, -1, dtype=np.int64)
    val[:L0] = init
    src_pos = (start[:, None] + np.arange(m_attach)[None, :]).ravel()
    val[src_pos] = np.repeat(newv, m_attach)
    tgt_pos = (start[:, None] + m_attach + np.arange(m_attach)[None, :]).ravel()
    ptr = np.floor(rng.random(tgt_pos.size) * np.repeat(start, m_attach)).astype(np.int64)
    # pointer jumping: a pointer to a target slot is replaced by that slot's pointer
    slot_ptr = np.full(total, -1, dtype=np.int64)
    slot_ptr[tgt_pos] = ptr
    for _ in range(64):
        nxt = slot_ptr[ptr]
        hop = nxt >= 0
        if not hop.any():
            break
        ptr = np.where(hop, nxt, ptr)
        slot_ptr[tgt_pos] = ptr
    tgt = val[ptr]
    assert (tgt >= 0).all()
    su = np.concatenate([iu.astype(np.int64), np.repeat(newv, m_attach)])
    sv = np.concatenate([iv.astype(np.int64), tgt])
    return su, sv


def ba_cliques(n: int, m_attach: int, num_cliques: int = 5, clique_size=(8, 20),
               seed=0) -> Graph:
    """Barabasi-Albert graph plus planted cliques, each on a uniformly chosen
    vertex subset of size drawn uniformly from clique_size (inclusive)."""
    rng = _rng(seed)
    u, v = barabasi_albert(n, m_attach, rng=rng)
    us, vs = [u], [v]
    sizes = []
    for _ in range(num_cliques):
        s = int(rng.integers(clique_size[0], clique_size[1] + 1))
        s = min(s, n)
        sizes.append(s)
        verts = rng.choice(n, size=s, replace=False)
        a, b = np.triu_indices(s, 1)
        us.append(verts[a])
        vs.append(verts[b])
    return from_edges(n, np.concatenate(us), np.concatenate(vs),
                      name=f"BA({n},{m_attach})+cliques",
                      meta={"seed": seed, "gen": "ba_cliques", "m_attach": m_attach,
                            "cliques": sizes})
