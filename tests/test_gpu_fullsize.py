"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (graph-driven rounds, default tuning, workspace reused): the oracle
cannot decompose these graphs in test time, so the GPU's (t, rho) is checked
with the oracle's exactness certificate -- every edge for the round/level
structure (C0), a sample of edges for the two support conditions (C1, C2) --
and against properties that hold at any size."""
import numpy as np
import pytest

from graphgen import workloads as W
from tests.gpu_helpers import assert_certified

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _decompose_like_bench(g, h):
    import torch
    import paper_2411_06405_amd as ht
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr.view(np.int32)).to(dev)
    ci = torch.from_numpy(g.col_idx.view(np.int32)).to(dev)
    ws = ht.alloc_workspace(g.n, g.m, h, device=dev)
    print(f"[gpu] {g.name} n={g.n} m={g.m} h={h} (bench configuration)", flush=True)
    t, rho = ht.decompose(rp, ci, g.n, h, workspace=ws, device=dev)
    st = ht.last_stats()
    sup = ht.h_support(rp, ci, g.n, h, workspace=ws, device=dev)
    out = (ht.to_numpy_u32(t), ht.to_numpy_u32(rho), ht.to_numpy_u32(sup), st)
    del ws
    torch.cuda.empty_cache()
    return out


def _check_any_size(t, rho, sup, st):
    # properties at any size: 2 <= t <= sup_G + 2; rounds numbered 0..R-1
    assert t.min() >= 2 and np.all(t <= sup.astype(np.int64) + 2)
    assert int(rho.max()) + 1 == st["rounds"]
    assert np.unique(rho).size == st["rounds"]


@pytest.mark.parametrize("make,h,nsample", [
    (lambda: W.d2(), 2, 3000),          # Chung-Lu n = 100,000
    (lambda: W.d3(), 2, 2000),          # R-MAT scale 18, h = 2 (the bench workload)
    (lambda: W.d3(), 3, 2000),          # R-MAT scale 18, h = 3
], ids=["chung_lu_100k_h2", "rmat18_h2", "rmat18_h3"])
def test_fullsize_certified(make, h, nsample):
    # C0 on every edge; C1 and C2 on nsample uniform edges plus the edges of
    # the first and last round and of the lowest and highest trussness
    g = make()
    t, rho, sup, st = _decompose_like_bench(g, h)
    _check_any_size(t, rho, sup, st)
    n = assert_certified(g, h, t, rho, nsample)
    print(f"[gpu] certified {n} sampled edges, {st['rounds']} rounds", flush=True)


@pytest.mark.parametrize("scale", [12, 13, 14])
def test_rmat_h3_fully_certified(scale):
    # R-MAT of the bench's parameters at scales the certificate covers edge by
    # edge: C0, C1 and C2 on every edge, so t is exact everywhere (Def. 4)
    import os
    import oracle
    g = W.d3(scale=scale)
    t, rho, sup, st = _decompose_like_bench(g, 3)
    _check_any_size(t, rho, sup, st)
    ok, fail = oracle.certify(g, 3, t, rho, sample=None,
                              threads=len(os.sched_getaffinity(0)))
    assert ok, f"R-MAT {scale} h=3: certificate check {fail}"
    print(f"[gpu] certified all {g.m} edges, {st['rounds']} rounds", flush=True)


# Serving size classes (Chung-Lu, n in {50k, 200k}), each the first request of
# its class and h in the seeded request stream
D5_CLASS_REQUESTS = {"n50k_h3": 27, "n50k_h4": 5, "n200k_h2": 4, "n200k_h3": 24}


@pytest.mark.parametrize("which", sorted(D5_CLASS_REQUESTS))
def test_serving_classes_certified(which):
    spec = W.d5_request_specs(200)[D5_CLASS_REQUESTS[which]]
    g = W.d5_graph(spec)
    h = spec[3]
    t, rho, sup, st = _decompose_like_bench(g, h)
    _check_any_size(t, rho, sup, st)
    n = assert_certified(g, h, t, rho, 2000)
    print(f"[gpu] {which}: certified {n} sampled edges, {st['rounds']} rounds", flush=True)


def test_fullsize_initial_support_sampled():
    # the initial h-support of sampled edges of the full Chung-Lu graph
    # against the oracle's BFS, edge by edge
    import oracle
    g = W.d2()
    _, _, sup, _ = _decompose_like_bench(g, 2)
    rng = np.random.default_rng(1)
    sample = rng.choice(g.m, 500, replace=False)
    ref = oracle.h_support_edges(g, 2, sample.astype(np.uint32))
    assert np.array_equal(sup[sample], ref)


def test_fullsize_hindex_equals_certified_peeling():
    # the H-index fixpoint method (Section 4) at the bench size and launch
    # configuration, synchronous and asynchronous, against the peeling
    # method's trussness, which the oracle's certificate checks here too
    import torch
    import paper_2411_06405_amd as ht
    g = W.d2()
    h = 2
    t, rho, _, _ = _decompose_like_bench(g, h)
    assert_certified(g, h, t, rho, 1000)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr.view(np.int32)).to(dev)
    ci = torch.from_numpy(g.col_idx.view(np.int32)).to(dev)
    ws = ht.hindex_workspace(rp, ci, g.n, h, device=dev)
    for asynchronous in (False, True):
        print(f"[gpu] H-index {g.name} h={h} asynchronous={asynchronous}", flush=True)
        th, sweeps = ht.hindex(rp, ci, g.n, h, asynchronous=asynchronous, workspace=ws, device=dev)
        th = ht.to_numpy_u32(th)
        bad = np.nonzero(th != t)[0]
        assert bad.size == 0, f"{bad.size} mismatches, first {bad[:5]}"
        assert 1 <= sweeps < 100
    del ws
    torch.cuda.empty_cache()
