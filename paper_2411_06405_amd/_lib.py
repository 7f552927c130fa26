"""ctypes binding of libhotruss (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; this module
only allocates device tensors with torch (outputs and the workspace), passes
raw device pointers and the current HIP stream, and translates status codes.
There is no CPU fallback: if the library is not built, importing fails.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np
import torch

LIB_PATH = Path(__file__).resolve().parent / "libhotruss.so"

HO_OK = 0
STATUS = {0: "HO_OK", -1: "HO_ERR_INVALID_ARG", -2: "HO_ERR_BAD_CSR", -3: "HO_ERR_WORKSPACE",
          -4: "HO_ERR_HIP", -5: "HO_ERR_BUDGET", -6: "HO_ERR_CANCELLED", -7: "HO_ERR_BUSY",
          -8: "HO_ERR_NOT_FOUND", -9: "HO_ERR_INTERNAL"}
HO_FLAG_HOST_LOOP = 0x1
HO_FLAG_STATS = 0x2
HO_FLAG_SERIAL_LEVELS = 0x4
HO_FLAG_SERIAL_SUPPORT = 0x8


class HotrussError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}")


class Tuning(C.Structure):
    _fields_ = [("word_bits", C.c_uint32), ("dense_threshold", C.c_uint32),
                ("edges_per_wave", C.c_uint32), ("flags", C.c_uint32),
                ("event_capacity", C.c_uint32), ("grid_blocks", C.c_uint32),
                ("item_capacity", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [("rounds", C.c_uint64), ("levels", C.c_uint64), ("events", C.c_uint64),
                ("overflows", C.c_uint64), ("device_ms", C.c_double),
                ("kernel_ms", C.c_double * 6), ("kernel_launches", C.c_uint64 * 6),
                ("work", C.c_uint64 * 8)]


KERNEL_KINDS = ("support_init", "jump_min", "mark", "level_events", "support_update", "advance")
WORK_KINDS = ("level_items", "level_slots", "level_candidates", "level_probes", "level_drops",
              "support_items", "support_slots", "support_hits")


def _declare(lib):
    vp, u32, u64, sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_size_t
    tp = C.POINTER(Tuning)
    lib.hoTrussWorkspaceBytes.argtypes = [u32, u64, u32, tp]
    lib.hoTrussWorkspaceBytes.restype = sz
    lib.hoTrussHSupport.argtypes = [vp, vp, u32, u64, u32, vp, vp, sz, tp, vp]
    lib.hoTrussHSupport.restype = C.c_int
    lib.hoTrussDecompose.argtypes = [vp, vp, u32, u64, u32, vp, vp, vp, sz, tp, vp]
    lib.hoTrussDecompose.restype = C.c_int
    lib.hoTrussLastStats.argtypes = [C.POINTER(Stats)]
    lib.hoTrussLastStats.restype = C.c_int
    lib.hoStatusString.argtypes = [C.c_int]
    lib.hoStatusString.restype = C.c_char_p
    if hasattr(lib, "hoTrussBatchedWorkspaceBytes"):
        lib.hoTrussBatchedWorkspaceBytes.argtypes = [vp, vp, vp, u32, tp]
        lib.hoTrussBatchedWorkspaceBytes.restype = sz
        lib.hoTrussDecomposeBatched.argtypes = [vp, vp, vp, vp, vp, vp, u32, vp, vp, vp, sz,
                                                tp, vp]
        lib.hoTrussDecomposeBatched.restype = C.c_int
    return lib


def load():
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    return _declare(C.CDLL(str(LIB_PATH)))


lib = load()

EXPORTS = ["hoStatusString", "hoTrussWorkspaceBytes", "hoTrussHSupport", "hoTrussDecompose",
           "hoTrussLastStats", "hoTrussBatchedWorkspaceBytes", "hoTrussDecomposeBatched"]


def _check(rc: int, what: str):
    if rc != HO_OK:
        raise HotrussError(rc, what)


def _tuning(tune):
    if tune is None:
        return None
    if isinstance(tune, Tuning):
        return C.byref(tune)
    t = Tuning(**tune)
    return C.byref(t)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_u32(a, device) -> torch.Tensor:
    """Device int32 tensor holding the bits of a uint32 array (no copy if already there)."""
    if isinstance(a, torch.Tensor):
        assert a.dtype in (torch.int32, torch.uint32) and a.is_contiguous()
        return a if a.device.type == "cuda" else a.to(device)
    arr = np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)
    return torch.from_numpy(arr).to(device)


def workspace_bytes(n: int, m: int, h: int, tune=None) -> int:
    return int(lib.hoTrussWorkspaceBytes(n, m, h, _tuning(tune)))


def alloc_workspace(n: int, m: int, h: int, tune=None, device="cuda") -> torch.Tensor:
    nb = workspace_bytes(n, m, h, tune)
    if nb == 0:
        raise HotrussError(-1, "hoTrussWorkspaceBytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def h_support(row_ptr, col_idx, n: int, h: int, workspace=None, tune=None, stream=None,
              device="cuda") -> torch.Tensor:
    """sup_G(e,h) of every edge (device int32 tensor holding uint32 values)."""
    rp = _dev_u32(row_ptr, device)
    ci = _dev_u32(col_idx, device)
    m = ci.numel() // 2
    out = torch.empty(max(m, 1), dtype=torch.int32, device=device)
    ws = workspace if workspace is not None else alloc_workspace(n, m, h, tune, device)
    rc = lib.hoTrussHSupport(rp.data_ptr(), ci.data_ptr(), n, m, h, out.data_ptr(),
                             ws.data_ptr(), ws.numel(), _tuning(tune), _stream(stream))
    _check(rc, "hoTrussHSupport")
    return out[:m]


def decompose(row_ptr, col_idx, n: int, h: int, with_rounds: bool = True, workspace=None,
              tune=None, stream=None, device="cuda"):
    """h-trussness (and peel round) of every edge: (t, rho) device int32 tensors."""
    rp = _dev_u32(row_ptr, device)
    ci = _dev_u32(col_idx, device)
    m = ci.numel() // 2
    t = torch.empty(max(m, 1), dtype=torch.int32, device=device)
    rho = torch.empty(max(m, 1), dtype=torch.int32, device=device) if with_rounds else None
    ws = workspace if workspace is not None else alloc_workspace(n, m, h, tune, device)
    rc = lib.hoTrussDecompose(rp.data_ptr(), ci.data_ptr(), n, m, h, t.data_ptr(),
                              rho.data_ptr() if rho is not None else None,
                              ws.data_ptr(), ws.numel(), _tuning(tune), _stream(stream))
    _check(rc, "hoTrussDecompose")
    return t[:m], (rho[:m] if rho is not None else None)


def last_stats() -> dict:
    s = Stats()
    _check(lib.hoTrussLastStats(C.byref(s)), "hoTrussLastStats")
    return {"rounds": s.rounds, "levels": s.levels, "events": s.events,
            "overflows": s.overflows, "device_ms": s.device_ms,
            "kernel_ms": dict(zip(KERNEL_KINDS, list(s.kernel_ms))),
            "kernel_launches": dict(zip(KERNEL_KINDS, list(s.kernel_launches))),
            "work": dict(zip(WORK_KINDS, list(s.work)))}


def to_numpy_u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def decompose_graph(g, h: int, **kw):
    """Convenience for host graphs (graphgen.Graph): returns numpy (t, rho)."""
    t, rho = decompose(g.row_ptr, g.col_idx, g.n, h, **kw)
    return to_numpy_u32(t), (to_numpy_u32(rho) if rho is not None else None)


def h_support_graph(g, h: int, **kw) -> np.ndarray:
    return to_numpy_u32(h_support(g.row_ptr, g.col_idx, g.n, h, **kw))
