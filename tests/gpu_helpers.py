"""Shared helpers of the GPU tests: run the HIP path, compare with the oracle."""
import numpy as np

import oracle


def run_gpu(g, h, **kw):
    import paper_2411_06405_amd as ht
    print(f"[gpu] {g.name} n={g.n} m={g.m} h={h} {kw}", flush=True)
    return ht.decompose_graph(g, h, **kw)


def assert_exact(g, h, **kw):
    t, rho = run_gpu(g, h, **kw)
    to, ro, info = oracle.decompose(g, h)
    bad = np.nonzero(t != to)[0]
    assert bad.size == 0, f"{g.name} h={h}: {bad.size} trussness mismatches, first {bad[:5]} " \
                          f"gpu {t[bad[:5]]} oracle {to[bad[:5]]}"
    assert np.array_equal(rho, ro), f"{g.name} h={h}: round schedule differs"
    return t, rho, info


def certificate_sample(t, rho, n: int, seed: int = 0) -> np.ndarray:
    """Edges whose exactness certificate is checked when the oracle cannot
    decompose the whole graph: n uniform edges, the edges of the first and the
    last peel round, and the edges of the lowest and highest trussness."""
    rng = np.random.default_rng(seed)
    m = t.size
    parts = [rng.choice(m, size=min(n, m), replace=False)]
    for mask in (rho == rho.min(), rho == rho.max(), t == t.min(), t == t.max()):
        idx = np.nonzero(mask)[0]
        parts.append(idx[:64] if idx.size <= 64 else rng.choice(idx, 64, replace=False))
    return np.unique(np.concatenate(parts)).astype(np.uint32)


def assert_certified(g, h, t, rho, n: int, seed: int = 0):
    """Certificate of (t, rho): C0 on every edge, C1 and C2 on a sample."""
    import os
    s = certificate_sample(t, rho, n, seed)
    ok, fail = oracle.certify(g, h, t, rho, sample=s, threads=len(os.sched_getaffinity(0)))
    assert ok, f"{g.name} h={h}: certificate check {fail}"
    return s.size
