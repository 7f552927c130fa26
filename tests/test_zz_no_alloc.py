"""The allocation-free entry point (hoTrussDecomposeNoAlloc) against the
plain one (hoTrussDecompose), through the C ABI: identical trussness and
round schedule on two calls in a row, the second on a smaller graph (the
fixed device array keeps the first call's contents), plus its size limit."""
import numpy as np
import pytest

from graphgen import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(g, h):
    import torch
    import paper_2411_06405_amd as ht
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr.view(np.int32)).to(dev)
    ci = torch.from_numpy(g.col_idx.view(np.int32)).to(dev)
    print(f"[gpu] no-alloc {g.name} n={g.n} m={g.m} h={h}", flush=True)
    t1, r1 = ht.decompose_noalloc(rp, ci, g.n, h, device=dev)
    st = ht.last_stats()
    t0, r0 = ht.decompose(rp, ci, g.n, h, device=dev)
    torch.cuda.synchronize()
    return (ht.to_numpy_u32(t1), ht.to_numpy_u32(r1), ht.to_numpy_u32(t0),
            ht.to_numpy_u32(r0), st)


def test_noalloc_equals_plain_two_calls_smaller_second():
    for g, h in ((W.d2(n=3000), 2), (W.d1(1), 2), (W.d3(scale=9), 3), (W.d1(2), 1)):
        t1, r1, t0, r0, st = _both(g, h)
        assert np.array_equal(t1, t0), f"{g.name} h={h}: trussness differs"
        assert np.array_equal(r1, r0), f"{g.name} h={h}: round schedule differs"
        assert st["rounds"] == int(r0.max()) + 1


def test_noalloc_rejects_graphs_beyond_its_array():
    import torch
    import paper_2411_06405_amd as ht
    g = W.d2(n=60000)  # balls alone need about 1.3 GB at h = 2
    with pytest.raises(ht.HotrussError) as ex:
        ht.decompose_noalloc(g.row_ptr, g.col_idx, g.n, 2, device=torch.device("cuda:0"))
    assert ex.value.status == -3
