"""ctypes shim over the plain C oracle (``hotruss_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Host numpy arrays in,
host numpy arrays out.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "hotruss_oracle.c"
_LIB = _HERE / "libhotruss_oracle.so"
_lib = None

OR_OK, OR_ERR_ARG, OR_ERR_CSR, OR_ERR_MEM, OR_CERT_FAIL = 0, -1, -2, -3, -10

class OracleError(RuntimeError):
    pass

def lib_path() -> Path:
    return _LIB

def build(force: bool = True) -> Path:
    """Compile the oracle with gcc + OpenMP (host code only)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
               str(_SRC), "-o", str(tmp)]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB

def _bind(path):
    """Load a compiled oracle and declare its entry points."""
    lib = C.CDLL(str(path))
    u32p = C.POINTER(C.c_uint32)
    u64p = C.POINTER(C.c_uint64)
    lib.oracle_h_support.argtypes = [C.c_uint32, u32p, u32p, C.c_uint32, u32p,
                                     C.c_uint32, u32p, C.c_int]
    lib.oracle_h_support_edges.argtypes = [C.c_uint32, u32p, u32p, C.c_uint32, u32p,
                                           C.c_uint32, u32p, C.c_uint64, u32p, C.c_int]
    lib.oracle_decompose.argtypes = [C.c_uint32, u32p, u32p, C.c_uint32, u32p, u32p,
                                     u32p, u32p, C.c_uint64, u64p, C.c_int]
    lib.oracle_certify.argtypes = [C.c_uint32, u32p, u32p, C.c_uint32, u32p, u32p,
                                   u32p, C.c_uint64, u64p, C.c_int]
    for f in (lib.oracle_h_support, lib.oracle_h_support_edges, lib.oracle_decompose,
              lib.oracle_certify):
        f.restype = C.c_int
    return lib

def compile_variant(src_text: str, out_path) -> "C.CDLL":
    """Compile an edited copy of the oracle source (used by the tests that
    plant a mistake in the oracle to show the pins catch it)."""
    out_path = Path(out_path)
    src = out_path.with_suffix(".c")
    src.write_text(src_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                    str(src), "-o", str(out_path)], check=True)
    return _bind(out_path)

def source_text() -> str:
    return _SRC.read_text()

def _load(lib=None):
    global _lib
    if lib is not None:
        return lib
    if _lib is None:
        if not _LIB.exists():
            build(force=False)
        _lib = _bind(_LIB)
    return _lib

def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(C.POINTER(C.c_uint32))

def _csr(g):
    rp, rpp = _u32(g.row_ptr)
    ci, cip = _u32(g.col_idx)
    return rp, rpp, ci, cip

def h_support(g, h: int, key=None, thr: int = 0, threads: int = 0, lib=None) -> np.ndarray:
    """sup_S(e,h) for every canonical edge, S = {f : key[f] >= thr} (all if key is None)."""
    lib = _load(lib)
    rp, rpp, ci, cip = _csr(g)
    out = np.zeros(g.m, dtype=np.uint32)
    kp = None
    if key is not None:
        key, kp = _u32(key)
    rc = lib.oracle_h_support(g.n, rpp, cip, int(h), kp, int(thr),
                              out.ctypes.data_as(C.POINTER(C.c_uint32)), int(threads))
    if rc != OR_OK:
        raise OracleError(f"oracle_h_support failed: {rc}")
    return out

def h_support_edges(g, h: int, edges, key=None, thr: int = 0, threads: int = 0,
                    lib=None) -> np.ndarray:
    """sup_S(e,h) for the listed canonical edges only (S as in h_support)."""
    lib = _load(lib)
    rp, rpp, ci, cip = _csr(g)
    edges, ep = _u32(edges)
    out = np.zeros(edges.size, dtype=np.uint32)
    kp = None
    if key is not None:
        key, kp = _u32(key)
    rc = lib.oracle_h_support_edges(g.n, rpp, cip, int(h), kp, int(thr), ep, edges.size,
                                    out.ctypes.data_as(C.POINTER(C.c_uint32)), int(threads))
    if rc != OR_OK:
        raise OracleError(f"oracle_h_support_edges failed: {rc}")
    return out


def decompose(g, h: int, threads: int = 0, round_cap: int = 1 << 20, lib=None):
    """Return (t, rho, info) with info = {rounds, levels, evals, round_k, round_size}."""
    lib = _load(lib)
    rp, rpp, ci, cip = _csr(g)
    m = g.m
    t = np.zeros(m, dtype=np.uint32)
    rho = np.zeros(m, dtype=np.uint32)
    cap = int(min(round_cap, max(m, 1)))
    rk = np.zeros(cap, dtype=np.uint32)
    rs = np.zeros(cap, dtype=np.uint32)
    st = np.zeros(4, dtype=np.uint64)
    P = C.POINTER(C.c_uint32)
    rc = lib.oracle_decompose(g.n, rpp, cip, int(h), t.ctypes.data_as(P), rho.ctypes.data_as(P),
                              rk.ctypes.data_as(P), rs.ctypes.data_as(P), cap,
                              st.ctypes.data_as(C.POINTER(C.c_uint64)), int(threads))
    if rc != OR_OK:
        raise OracleError(f"oracle_decompose failed: {rc}")
    R = int(st[0])
    info = {"rounds": R, "levels": int(st[1]), "evals": int(st[2]),
            "round_k": rk[:min(R, cap)].copy(), "round_size": rs[:min(R, cap)].copy()}
    return t, rho, info

def certify(g, h: int, t, rho, sample=None, threads: int = 0, lib=None):
    """Check the exactness certificate of (t, rho); returns (ok, fail_info)."""
    lib = _load(lib)
    rp, rpp, ci, cip = _csr(g)
    t, tp = _u32(t)
    rho, rhop = _u32(rho)
    sp, ns = None, 0
    if sample is not None:
        sample, sp = _u32(sample)
        ns = sample.size
    fail = np.zeros(3, dtype=np.uint64)
    rc = lib.oracle_certify(g.n, rpp, cip, int(h), tp, rhop, sp, ns,
                            fail.ctypes.data_as(C.POINTER(C.c_uint64)), int(threads))
    if rc == OR_OK:
        return True, None
    if rc == OR_CERT_FAIL:
        return False, {"check": int(fail[0]), "edge": int(fail[1]), "value": int(fail[2])}
    raise OracleError(f"oracle_certify failed: {rc}")
