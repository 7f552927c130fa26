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
HO_ERR_WORKSPACE = -3
STATUS = {0: "HO_OK", -1: "HO_ERR_INVALID_ARG", -2: "HO_ERR_BAD_CSR", -3: "HO_ERR_WORKSPACE",
          -4: "HO_ERR_HIP", -5: "HO_ERR_BUDGET", -6: "HO_ERR_CANCELLED", -7: "HO_ERR_BUSY",
          -8: "HO_ERR_NOT_FOUND", -9: "HO_ERR_INTERNAL"}
HO_FLAG_HOST_LOOP = 0x1
HO_FLAG_STATS = 0x2
HO_FLAG_SERIAL_LEVELS = 0x4
HO_FLAG_SERIAL_SUPPORT = 0x8
HO_FLAG_COMPACT_EACH = 0x10


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
                ("overflows", C.c_uint64), ("compactions", C.c_uint64),
                ("device_ms", C.c_double),
                ("kernel_ms", C.c_double * 6), ("kernel_launches", C.c_uint64 * 6),
                ("work", C.c_uint64 * 8), ("evaluations", C.c_uint64),
                ("alg_bytes", C.c_uint64), ("level_events", C.c_uint64 * 16)]


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
    lib.hoTrussDecomposeNoAlloc.argtypes = [vp, vp, u32, u64, u32, vp, vp, vp]
    lib.hoTrussDecomposeNoAlloc.restype = C.c_int
    lib.hoTrussLastStats.argtypes = [C.POINTER(Stats)]
    lib.hoTrussLastStats.restype = C.c_int
    lib.hoStatusString.argtypes = [C.c_int]
    lib.hoStatusString.restype = C.c_char_p
    lib.hoTrussBatchedWorkspaceBytes.argtypes = [vp, vp, vp, u32, tp]
    lib.hoTrussBatchedWorkspaceBytes.restype = sz
    lib.hoTrussDecomposeBatched.argtypes = [vp, vp, vp, vp, vp, vp, u32, vp, vp, vp, sz, tp, vp]
    lib.hoTrussDecomposeBatched.restype = C.c_int
    lib.hoSessionCreate.argtypes = [vp, sz, u32, u32, vp, C.POINTER(vp)]
    lib.hoSessionCreate.restype = C.c_int
    lib.hoSubmit.argtypes = [vp, vp, vp, u32, u64, u32, vp, vp, C.POINTER(u64)]
    lib.hoSubmit.restype = C.c_int
    lib.hoSessionProgress.argtypes = [vp, u32, C.POINTER(u32), C.POINTER(u32)]
    lib.hoSessionProgress.restype = C.c_int
    lib.hoPoll.argtypes = [vp, u64, C.POINTER(C.c_int)]
    lib.hoPoll.restype = C.c_int
    lib.hoCancel.argtypes = [vp, u64]
    lib.hoCancel.restype = C.c_int
    lib.hoSessionDestroy.argtypes = [vp]
    lib.hoTrussComponentsWorkspaceBytes.argtypes = [u32, u64]
    lib.hoTrussComponentsWorkspaceBytes.restype = sz
    lib.hoTrussComponents.argtypes = [vp, vp, u32, u64, vp, u32, vp, C.POINTER(u32), vp, sz, vp]
    lib.hoTrussComponents.restype = C.c_int
    lib.hoSessionDestroy.restype = C.c_int
    lib.hoTrussHIndexWorkspaceBytes.argtypes = [u32, u64, u32]
    lib.hoTrussHIndexWorkspaceBytes.restype = sz
    lib.hoTrussHIndex.argtypes = [vp, vp, u32, u64, u32, u32, u32, vp, C.POINTER(u32), vp, sz,
                                  C.POINTER(sz), vp]
    lib.hoTrussHIndex.restype = C.c_int
    return lib


def load():
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    return _declare(C.CDLL(str(LIB_PATH)))


lib = load()

EXPORTS = ["hoStatusString", "hoTrussWorkspaceBytes", "hoTrussHSupport", "hoTrussDecompose",
           "hoTrussDecomposeNoAlloc",
           "hoTrussLastStats", "hoTrussBatchedWorkspaceBytes", "hoTrussDecomposeBatched",
           "hoSessionCreate", "hoSubmit", "hoSessionProgress", "hoPoll", "hoCancel",
           "hoSessionDestroy", "hoTrussComponentsWorkspaceBytes", "hoTrussComponents",
           "hoTrussHIndexWorkspaceBytes", "hoTrussHIndex"]

HO_HINDEX_ASYNC = 0x1
HO_HINDEX_ALL = 0x2
HO_HINDEX_STATS = 0x4
HO_HINDEX_KEYS = 0x8


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


def decompose_noalloc(row_ptr, col_idx, n: int, h: int, out_trussness=None, out_round=None,
                      stream=None, device="cuda"):
    """hoTrussDecomposeNoAlloc: the library allocates nothing (its workspace
    is a fixed device array inside the library).  Outputs may be passed in;
    otherwise this binding allocates them."""
    rp = _dev_u32(row_ptr, device)
    ci = _dev_u32(col_idx, device)
    m = ci.numel() // 2
    t = out_trussness if out_trussness is not None else \
        torch.empty(max(m, 1), dtype=torch.int32, device=device)
    rho = out_round if out_round is not None else \
        torch.empty(max(m, 1), dtype=torch.int32, device=device)
    rc = lib.hoTrussDecomposeNoAlloc(rp.data_ptr(), ci.data_ptr(), n, m, h, t.data_ptr(),
                                     rho.data_ptr(), _stream(stream))
    _check(rc, "hoTrussDecomposeNoAlloc")
    return t[:m], rho[:m]


def last_stats() -> dict:
    s = Stats()
    _check(lib.hoTrussLastStats(C.byref(s)), "hoTrussLastStats")
    return {"rounds": s.rounds, "levels": s.levels, "events": s.events,
            "overflows": s.overflows, "compactions": s.compactions, "device_ms": s.device_ms,
            "kernel_ms": dict(zip(KERNEL_KINDS, list(s.kernel_ms))),
            "kernel_launches": dict(zip(KERNEL_KINDS, list(s.kernel_launches))),
            "work": dict(zip(WORK_KINDS, list(s.work))),
            "evaluations": s.evaluations, "alg_bytes": s.alg_bytes,
            "level_events": list(s.level_events)}


def to_numpy_u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def decompose_graph(g, h: int, **kw):
    """Convenience for host graphs (graphgen.Graph): returns numpy (t, rho)."""
    t, rho = decompose(g.row_ptr, g.col_idx, g.n, h, **kw)
    return to_numpy_u32(t), (to_numpy_u32(rho) if rho is not None else None)


def h_support_graph(g, h: int, **kw) -> np.ndarray:
    return to_numpy_u32(h_support(g.row_ptr, g.col_idx, g.n, h, **kw))


def hindex_workspace(row_ptr, col_idx, n: int, h: int, pruning: str = "lemma4", stream=None,
                     device="cuda"):
    """A workspace that fits this graph's H-index run (two calls: the first
    reports the size the balls need)."""
    if pruning not in ("lemma4", "keys"):
        raise ValueError("pruning is 'lemma4' (the paper's rule on edge values) or 'keys'")
    rp = _dev_u32(row_ptr, device)
    ci = _dev_u32(col_idx, device)
    m = ci.numel() // 2
    nb = int(lib.hoTrussHIndexWorkspaceBytes(n, m, h))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
    if m == 0:
        return ws
    out = torch.empty(m, dtype=torch.int32, device=device)
    sweeps = C.c_uint32()
    needed = C.c_size_t()
    flags = HO_HINDEX_KEYS if pruning == "keys" else 0
    rc = lib.hoTrussHIndex(rp.data_ptr(), ci.data_ptr(), n, m, h, flags, 1, out.data_ptr(),
                           C.byref(sweeps), ws.data_ptr(), ws.numel(), C.byref(needed),
                           _stream(stream))
    if rc == HO_ERR_WORKSPACE and needed.value > ws.numel():
        return torch.empty(int(needed.value), dtype=torch.uint8, device=device)
    _check(rc, "hoTrussHIndex")
    return ws


def hindex(row_ptr, col_idx, n: int, h: int, asynchronous: bool = False, track: bool = True,
           max_sweeps: int = 0, workspace=None, stream=None, device="cuda", stats: bool = False,
           pruning: str = "lemma4"):
    """Trussness by the H-index fixpoint method: (t device tensor, sweeps).

    The workspace size depends on the h-hop balls, which only the device
    knows: a first call with the minimum reports the size needed; the
    workspace is then grown and the call repeated.  A caller-given workspace
    that is too small raises."""
    if pruning not in ("lemma4", "keys"):
        raise ValueError("pruning is 'lemma4' (the paper's rule on edge values) or 'keys'")
    rp = _dev_u32(row_ptr, device)
    ci = _dev_u32(col_idx, device)
    m = ci.numel() // 2
    out = torch.empty(max(m, 1), dtype=torch.int32, device=device)
    flags = ((HO_HINDEX_ASYNC if asynchronous else 0) | (0 if track else HO_HINDEX_ALL)
             | (HO_HINDEX_STATS if stats else 0) | (HO_HINDEX_KEYS if pruning == "keys" else 0))
    sweeps = C.c_uint32()
    needed = C.c_size_t()
    grow = workspace is None
    if grow:
        nb = int(lib.hoTrussHIndexWorkspaceBytes(n, m, h))
        workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
    for _ in range(2):
        rc = lib.hoTrussHIndex(rp.data_ptr(), ci.data_ptr(), n, m, h, flags, int(max_sweeps),
                               out.data_ptr(), C.byref(sweeps), workspace.data_ptr(),
                               workspace.numel(), C.byref(needed), _stream(stream))
        if rc == HO_ERR_WORKSPACE and grow and needed.value > workspace.numel():
            workspace = torch.empty(int(needed.value), dtype=torch.uint8, device=device)
            continue
        break
    _check(rc, "hoTrussHIndex")
    return out[:m], int(sweeps.value)


def hindex_graph(g, h: int, **kw):
    """Convenience for host graphs: numpy trussness and the sweep count."""
    t, sweeps = hindex(g.row_ptr, g.col_idx, g.n, h, **kw)
    return to_numpy_u32(t), sweeps


def truss_components(row_ptr, col_idx, n: int, trussness, k: int, workspace=None, stream=None,
                     device="cuda"):
    """(k,h)-truss extraction: (label per edge, number of components).

    label[e] (device int32 tensor holding uint32 values) is the smallest vertex
    of e's component among the edges with t(e) >= k, 0xFFFFFFFF below k."""
    rp = _dev_u32(row_ptr, device)
    ci = _dev_u32(col_idx, device)
    t = _dev_u32(trussness, device)
    m = ci.numel() // 2
    out = torch.empty(max(m, 1), dtype=torch.int32, device=device)
    if workspace is None:
        nb = int(lib.hoTrussComponentsWorkspaceBytes(n, m))
        workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
    count = C.c_uint32()
    rc = lib.hoTrussComponents(rp.data_ptr(), ci.data_ptr(), n, m, t.data_ptr(), int(k),
                               out.data_ptr(), C.byref(count), workspace.data_ptr(),
                               workspace.numel(), _stream(stream))
    _check(rc, "hoTrussComponents")
    return out[:m], int(count.value)


def truss_components_graph(g, trussness, k: int, **kw):
    """Convenience for host graphs: numpy uint32 labels and the count."""
    lab, c = truss_components(g.row_ptr, g.col_idx, g.n, trussness, k, **kw)
    return to_numpy_u32(lab), c


def _host_ptr(a: np.ndarray, dtype) -> tuple:
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr, arr.ctypes.data


def batched_workspace_bytes(vtx_off, edge_off, h, tune=None) -> int:
    vo, vop = _host_ptr(vtx_off, np.uint64)
    eo, eop = _host_ptr(edge_off, np.uint64)
    hh, hp = _host_ptr(h, np.uint32)
    return int(lib.hoTrussBatchedWorkspaceBytes(vop, eop, hp, hh.size, _tuning(tune)))


def decompose_batched(row_ptr_cat, col_idx_cat, vtx_off, adj_off, edge_off, h,
                      with_rounds: bool = True, workspace=None, tune=None, stream=None,
                      device="cuda"):
    """Batched decomposition of concatenated graphs (offset arrays on the host).

    Returns (t_cat, rho_cat) device int32 tensors in concatenated edge order."""
    rp = _dev_u32(row_ptr_cat, device)
    ci = _dev_u32(col_idx_cat, device)
    vo, vop = _host_ptr(vtx_off, np.uint64)
    ao, aop = _host_ptr(adj_off, np.uint64)
    eo, eop = _host_ptr(edge_off, np.uint64)
    hh, hp = _host_ptr(h, np.uint32)
    B = hh.size
    mt = int(eo[-1]) if B else 0
    t = torch.empty(max(mt, 1), dtype=torch.int32, device=device)
    rho = torch.empty(max(mt, 1), dtype=torch.int32, device=device) if with_rounds else None
    if workspace is None:
        nb = batched_workspace_bytes(vo, eo, hh, tune)
        workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
    rc = lib.hoTrussDecomposeBatched(rp.data_ptr(), ci.data_ptr(), vop, aop, eop, hp, B,
                                     t.data_ptr(), rho.data_ptr() if rho is not None else None,
                                     workspace.data_ptr(), workspace.numel(), _tuning(tune),
                                     _stream(stream))
    _check(rc, "hoTrussDecomposeBatched")
    return t[:mt], (rho[:mt] if rho is not None else None)


def decompose_batch(batch, **kw):
    """Convenience for graphgen.Batch: returns per-graph numpy (t, rho) lists."""
    t, rho = decompose_batched(batch.row_ptr_cat, batch.col_idx_cat, batch.vtx_off,
                               batch.adj_off, batch.edge_off, batch.h, **kw)
    tn = to_numpy_u32(t)
    rn = to_numpy_u32(rho) if rho is not None else None
    eo = batch.edge_off.astype(np.int64)
    ts = [tn[eo[g]:eo[g + 1]] for g in range(batch.B)]
    rs = [rn[eo[g]:eo[g + 1]] for g in range(batch.B)] if rn is not None else None
    return ts, rs


class Session:
    """Continuous-batching session over a device memory pool (hoSession*).

    submit() queues a graph whose device CSR and outputs the session keeps
    alive until the request is done; progress() admits and runs rounds."""

    def __init__(self, pool_bytes: int, max_slots: int = 64, max_h: int = 4, stream=None,
                 device="cuda"):
        self.device = device
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self._h = C.c_void_p()
        rc = lib.hoSessionCreate(self.pool.data_ptr(), pool_bytes, max_slots, max_h,
                                 _stream(stream), C.byref(self._h))
        _check(rc, "hoSessionCreate")
        self._keep = {}

    def submit(self, row_ptr, col_idx, n: int, h: int) -> int:
        rp = _dev_u32(row_ptr, self.device)
        ci = _dev_u32(col_idx, self.device)
        m = ci.numel() // 2
        t = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        rho = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        ticket = C.c_uint64()
        rc = lib.hoSubmit(self._h, rp.data_ptr(), ci.data_ptr(), n, m, h, t.data_ptr(),
                          rho.data_ptr(), C.byref(ticket))
        _check(rc, "hoSubmit")
        self._keep[ticket.value] = (rp, ci, t, rho, m)
        return ticket.value

    def progress(self, max_graph_launches: int = 0):
        a, q = C.c_uint32(), C.c_uint32()
        rc = lib.hoSessionProgress(self._h, max_graph_launches, C.byref(a), C.byref(q))
        _check(rc, "hoSessionProgress")
        return a.value, q.value

    def poll(self, ticket: int) -> bool:
        done = C.c_int()
        rc = lib.hoPoll(self._h, ticket, C.byref(done))
        _check(rc, "hoPoll")
        return bool(done.value)

    def status(self, ticket: int) -> int:
        done = C.c_int()
        return int(lib.hoPoll(self._h, ticket, C.byref(done)))

    def cancel(self, ticket: int) -> None:
        _check(lib.hoCancel(self._h, ticket), "hoCancel")

    def result(self, ticket: int):
        """(t, rho) numpy uint32 arrays of a finished request; releases its buffers."""
        if not self.poll(ticket):
            raise HotrussError(-7, "request not finished")
        rp, ci, t, rho, m = self._keep.pop(ticket)
        return to_numpy_u32(t[:m]), to_numpy_u32(rho[:m])

    def close(self):
        if self._h:
            _check(lib.hoSessionDestroy(self._h), "hoSessionDestroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
