"""hotruss: higher-order (k,h)-truss decomposition on AMD Instinct MI355X.

The computation lives in libhotruss.so (hand-written HIP kernels for gfx950,
C ABI declared in include/hotruss.h); this package is its thin Python binding.
"""
from . import autotune
from ._lib import (HotrussError, Session, Tuning, alloc_workspace, batched_workspace_bytes,
                   decompose, decompose_batch, decompose_batched, decompose_graph,
                   decompose_noalloc, h_support,
                   h_support_graph, hindex, hindex_graph, hindex_workspace, last_stats, lib, to_numpy_u32, truss_components,
                   truss_components_graph, workspace_bytes)

__all__ = ["autotune", "HotrussError", "Session", "Tuning", "alloc_workspace", "batched_workspace_bytes",
           "decompose", "decompose_batch", "decompose_batched", "decompose_graph",
           "decompose_noalloc", "h_support",
           "h_support_graph", "hindex", "hindex_graph", "hindex_workspace", "last_stats", "lib", "to_numpy_u32", "truss_components",
           "truss_components_graph", "workspace_bytes"]
