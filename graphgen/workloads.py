"""Named workload recipes (seeded), one per configuration the library is
measured and tested on.  Sizes and seeds are fixed here so that tests, the
benchmark and the golden-value script all see the same graphs.
"""
from __future__ import annotations

import numpy as np

from . import gen
from .csr import Graph

# uniform random graph, small enough for the plain CPU oracle (h = 2 headline)
D1_N, D1_P = 200, 0.05
D1_SEEDS = (0, 1, 2, 3, 4)

# power-law Chung-Lu, the single-graph throughput workload
D2_N, D2_DEG, D2_GAMMA, D2_SEED = 100_000, 10.0, 2.5, 1

# R-MAT scale 18, edge factor 16
D3_SCALE, D3_EF, D3_ABCD, D3_SEED = 18, 16, (0.57, 0.19, 0.19, 0.05), 1

# batched: preferential attachment plus planted cliques
D4_B, D4_NRANGE, D4_MRANGE, D4_CLIQUES, D4_CSIZE, D4_HS, D4_SEED = \
    512, (1_000, 50_000), (3, 8), 5, (8, 20), (2, 3), 7

# serving: Poisson stream over size classes
D5_NCLASSES = (500, 5_000, 50_000, 200_000)
D5_GAMMA, D5_DEG, D5_HS, D5_SEED = (2.1, 2.8), (6.0, 20.0), (2, 3, 4), 11


def d1(seed: int = 0) -> Graph:
    return gen.erdos_renyi(D1_N, D1_P, seed=seed)


def d2(n: int = D2_N, seed: int = D2_SEED) -> Graph:
    return gen.chung_lu(n, D2_DEG, D2_GAMMA, seed=seed)


def d3(scale: int = D3_SCALE, seed: int = D3_SEED) -> Graph:
    return gen.rmat(scale, D3_EF, D3_ABCD, seed=seed)


def d4_specs(B: int = D4_B, seed: int = D4_SEED, nrange=D4_NRANGE):
    """Per-graph (n, m_attach, h, graph_seed) for the batched workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(nrange[0], nrange[1] + 1, size=B)
    ms = rng.integers(D4_MRANGE[0], D4_MRANGE[1] + 1, size=B)
    hs = rng.choice(np.array(D4_HS), size=B)
    seeds = rng.integers(0, 2**31 - 1, size=B)
    return [(int(n), int(m), int(h), int(s)) for n, m, h, s in zip(ns, ms, hs, seeds)]


def d4_graph(spec) -> Graph:
    n, m, h, s = spec
    g = gen.ba_cliques(n, m, D4_CLIQUES, D4_CSIZE, seed=s)
    g.meta["h"] = h
    return g


def d5_request_specs(num: int, seed: int = D5_SEED, nclasses=D5_NCLASSES):
    """Per-request (n, gamma, avg_deg, h, graph_seed) for the serving stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(num):
        n = int(rng.choice(np.array(nclasses)))
        gamma = float(rng.uniform(*D5_GAMMA))
        deg = float(rng.uniform(*D5_DEG))
        h = int(rng.choice(np.array(D5_HS)))
        s = int(rng.integers(0, 2**31 - 1))
        out.append((n, gamma, deg, h, s))
    return out


def d5_graph(spec) -> Graph:
    n, gamma, deg, h, s = spec
    g = gen.chung_lu(n, deg, gamma, seed=s)
    g.meta["h"] = h
    return g


def poisson_arrivals(num: int, qps: float, seed: int = D5_SEED) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream at rate qps."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / qps, size=num))
