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
