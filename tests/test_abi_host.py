"""Host-only checks of the C ABI: the library loads, exports every entry point
include/hotruss.h declares, sizes workspaces sensibly and rejects bad
arguments before any device work (no GPU needed)."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "hotruss.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ho[A-Z]\w*)\s*\(", text)))


@pytest.fixture(scope="module")
def ht():
    import paper_2411_06405_amd as ht
    return ht


def test_exports_every_declared_symbol(ht):
    names = declared_functions()
    assert "hoTrussDecompose" in names and "hoTrussHSupport" in names
    for name in names:
        assert hasattr(ht.lib, name), name


def test_status_strings(ht):
    for code in range(0, -10, -1):
        s = ht.lib.hoStatusString(code)
        assert s and s != b"unknown status"


def test_workspace_query(ht):
    wb = ht.workspace_bytes
    assert wb(200, 1000, 0) == 0                       # h = 0 is invalid
    assert wb(200, 1000, 1) < wb(200, 1000, 2) < wb(200, 1000, 3)
    assert wb(1000, 5000, 2) > wb(500, 5000, 2)
    assert wb(10, 20, 100) == wb(10, 20, 9)             # h clamps at n-1
    assert wb(100, 1 << 31, 2) == 0                     # m too large
    # the ball store dominates: 2h bitset arrays of n x ceil(n/64) words
    n = 100_000
    rows = n * ((n + 63) // 64 + 7) // 8 * 8 * 8
    assert wb(n, 500_000, 2) >= 3 * rows


def test_argument_errors_return_before_device_work(ht):
    lib = ht.lib
    nul = None
    # h == 0
    assert lib.hoTrussDecompose(nul, nul, 10, 5, 0, nul, nul, nul, 0, nul, nul) == -1
    assert lib.hoTrussHSupport(nul, nul, 10, 5, 0, nul, nul, 0, nul, nul) == -1
    # NULL buffers with m > 0
    assert lib.hoTrussDecompose(nul, nul, 10, 5, 2, nul, nul, nul, 0, nul, nul) == -1
    # m == 0 is a no-op success
    assert lib.hoTrussDecompose(nul, nul, 10, 0, 2, nul, nul, nul, 0, nul, nul) == 0
    # workspace too small (pointers non-NULL but never dereferenced)
    fake = C.c_void_p(0x1000)
    assert lib.hoTrussDecompose(fake, fake, 10, 5, 2, fake, nul, fake, 16, nul, nul) == -3
    assert lib.hoTrussHSupport(fake, fake, 10, 5, 2, fake, fake, 16, nul, nul) == -3
    s = ht._lib.Stats()
    assert lib.hoTrussLastStats(None) == -1
    assert lib.hoTrussLastStats(C.byref(s)) == 0


def test_batched_argument_errors_return_before_device_work(ht):
    import numpy as np
    lib = ht.lib
    nul = None
    fake = C.c_void_p(0x1000)
    vo = np.array([0, 10, 30], dtype=np.uint64)
    ao = np.array([0, 20, 60], dtype=np.uint64)
    eo = np.array([0, 10, 30], dtype=np.uint64)
    h = np.array([2, 3], dtype=np.uint32)
    P = lambda a: a.ctypes.data  # noqa: E731
    # no graphs: a no-op success; missing offset arrays: invalid
    assert lib.hoTrussDecomposeBatched(nul, nul, P(vo), P(ao), P(eo), P(h), 0, nul, nul, nul,
                                       0, nul, nul) == 0
    assert lib.hoTrussDecomposeBatched(fake, fake, nul, P(ao), P(eo), P(h), 2, fake, nul, fake,
                                       1 << 30, nul, nul) == -1
    # h == 0 in one graph
    h0 = np.array([2, 0], dtype=np.uint32)
    assert lib.hoTrussDecomposeBatched(fake, fake, P(vo), P(ao), P(eo), P(h0), 2, fake, nul,
                                       fake, 1 << 30, nul, nul) == -1
    # adjacency and edge offsets disagree (2m_g != adj_off[g+1]-adj_off[g])
    bad = np.array([0, 20, 58], dtype=np.uint64)
    assert lib.hoTrussDecomposeBatched(fake, fake, P(vo), P(bad), P(eo), P(h), 2, fake, nul,
                                       fake, 1 << 30, nul, nul) == -1
    # workspace below the largest graph's share
    assert lib.hoTrussDecomposeBatched(fake, fake, P(vo), P(ao), P(eo), P(h), 2, fake, nul,
                                       fake, 4096, nul, nul) == -3


def test_batched_workspace_query(ht):
    import numpy as np
    # 100 equal graphs: the query covers the 64 largest at once, so it grows
    # with B up to 64 and not beyond
    def q(B, n=1000, m=4000, h=2):
        vo = np.arange(B + 1, dtype=np.uint64) * n
        eo = np.arange(B + 1, dtype=np.uint64) * m
        return ht.batched_workspace_bytes(vo, eo, np.full(B, h, np.uint32))
    one = ht.workspace_bytes(1000, 4000, 2)
    assert q(1) > 0
    assert q(1) < one  # smaller event and item lists than the plain path
    assert q(8) > 7 * q(1) // 2
    assert q(64) == q(100) or abs(q(64) - q(100)) < 1 << 20
    assert q(0) == 0


def test_session_argument_errors(ht):
    lib = ht.lib
    nul = None
    out = C.c_void_p()
    fake = C.c_void_p(0x1000)
    assert lib.hoSessionCreate(nul, 1 << 20, 4, 2, nul, C.byref(out)) == -1
    assert lib.hoSessionCreate(fake, 1 << 20, 0, 2, nul, C.byref(out)) == -1
    assert lib.hoSessionCreate(fake, 1 << 20, 4, 0, nul, C.byref(out)) == -1
    assert lib.hoSessionCreate(fake, 1 << 20, 4, 17, nul, C.byref(out)) == -1
    t = C.c_uint64()
    d = C.c_int()
    assert lib.hoSubmit(nul, fake, fake, 10, 5, 2, fake, nul, C.byref(t)) == -1
    assert lib.hoSessionProgress(nul, 0, nul, nul) == -1
    assert lib.hoPoll(nul, 0, C.byref(d)) == -1
    assert lib.hoCancel(nul, 0) == -1
    assert lib.hoSessionDestroy(nul) == -1


def test_hindex_argument_errors_return_before_device_work(ht):
    lib = ht.lib
    nul = None
    fake = C.c_void_p(0x1000)
    sw = C.c_uint32(7)
    need = C.c_size_t(0)
    args = lambda h, flags, ws_bytes, sweeps=C.byref(sw): (  # noqa: E731
        fake, fake, 10, 5, h, flags, 0, fake, sweeps, fake, ws_bytes, C.byref(need), nul)
    assert lib.hoTrussHIndex(*args(0, 0, 1 << 30)) == -1          # h == 0
    assert lib.hoTrussHIndex(*args(2, 16, 1 << 30)) == -1         # unknown flag
    assert lib.hoTrussHIndex(*args(2, 0, 1 << 30, None)) == -1    # no sweep count
    # workspace below the minimum: HO_ERR_WORKSPACE and the minimum reported
    assert lib.hoTrussHIndex(*args(2, 0, 16)) == -3
    assert need.value == lib.hoTrussHIndexWorkspaceBytes(10, 5, 2) > 16
    # m == 0: nothing to do
    assert lib.hoTrussHIndex(nul, nul, 10, 0, 2, 0, 0, nul, C.byref(sw), nul, 0, nul, nul) == 0
    assert sw.value == 0
    wb = lib.hoTrussHIndexWorkspaceBytes
    assert wb(200, 1000, 0) == 0
    assert wb(200, 1000, 1) < wb(200, 1000, 2) < wb(200, 1000, 3)
    assert wb(1000, 5000, 2) > wb(500, 5000, 2)


def test_binding_constants_match_the_header(ht):
    # every HO_* flag the binding passes has the value the header defines
    text = (ROOT / "include" / "hotruss.h").read_text()
    defined = {name: int(val, 16) for name, val in
               re.findall(r"#define\s+(HO_\w+)\s+(0x[0-9a-fA-F]+)u", text)}
    used = {name: getattr(ht._lib, name) for name in dir(ht._lib)
            if name.startswith(("HO_FLAG_", "HO_HINDEX_"))}
    assert used and set(used) <= set(defined)
    for name, val in used.items():
        assert defined[name] == val, name
    enum = dict((name, int(val)) for name, val in re.findall(r"(HO_\w+)\s*=\s*(-?\d+)", text))
    assert enum["HO_OK"] == ht._lib.HO_OK and enum["HO_ERR_WORKSPACE"] == ht._lib.HO_ERR_WORKSPACE


def test_hindex_binding_rejects_unknown_pruning_on_the_host(ht):
    import numpy as np
    rp = np.array([0, 1, 2], dtype=np.uint32)
    ci = np.array([1, 0], dtype=np.uint32)
    with pytest.raises(ValueError):
        ht.hindex(rp, ci, 2, 2, pruning="bogus")
    with pytest.raises(ValueError):
        ht.hindex_workspace(rp, ci, 2, 2, pruning="bogus")


def test_vertex_cap_of_the_ball_rows(ht):
    # a ball row (ceil(n/64) words, rounded up to 8) must fit the 64 KiB of
    # LDS a workgroup builds it in: n <= 524,288; above that every entry point
    # that keeps balls refuses before any device work
    lib = ht.lib
    cap = 524_288
    assert ht.workspace_bytes(cap, 1000, 2) > 0
    assert ht.workspace_bytes(cap + 1, 1000, 2) == 0
    assert lib.hoTrussHIndexWorkspaceBytes(cap, 1000, 2) > 0
    assert lib.hoTrussHIndexWorkspaceBytes(cap + 1, 1000, 2) == 0
    fake = C.c_void_p(0x1000)
    big = C.c_size_t(1 << 62)
    assert lib.hoTrussDecompose(fake, fake, cap + 1, 5, 2, fake, None, fake, big, None,
                                None) == -1
    assert lib.hoTrussHSupport(fake, fake, cap + 1, 5, 2, fake, fake, big, None, None) == -1


def test_noalloc_size_limit_before_device_work(ht):
    # the allocation-free entry point has a fixed 256 MiB device array: a graph
    # whose workspace does not fit is refused before any device work
    lib = ht.lib
    fake = C.c_void_p(0x1000)
    assert lib.hoTrussDecomposeNoAlloc(fake, fake, 60_000, 300_000, 2, fake, fake, None) == -3
    assert lib.hoTrussDecomposeNoAlloc(fake, fake, 524_289, 5, 2, fake, fake, None) == -1
    assert lib.hoTrussDecomposeNoAlloc(fake, fake, 10, 5, 0, fake, fake, None) == -1
    assert lib.hoTrussDecomposeNoAlloc(None, None, 10, 0, 2, None, None, None) == 0
