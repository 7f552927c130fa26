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
