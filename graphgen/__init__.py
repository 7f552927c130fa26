"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Input preparation only: no part of the truss computation lives here.
"""
from .csr import Batch, Graph, concat, disjoint_union, from_edge_list, from_edges, validate
from . import gen, workloads

__all__ = ["Batch", "Graph", "concat", "disjoint_union", "from_edge_list",
           "from_edges", "validate", "gen", "workloads"]
