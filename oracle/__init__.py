"""Plain CPU oracle for higher-order truss decomposition.

TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference that the GPU
library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
library (``paper_2411_06405_amd``) and never imports it.
"""
from .oracle import (OracleError, build, certify, decompose, h_support, h_support_edges,
                     lib_path)
from .brute import brute_trussness, brute_h_support
from .components import truss_components
from .hindex import hindex_sequence, hindex_trussness
from . import accounting

__all__ = ["OracleError", "build", "certify", "decompose", "h_support", "h_support_edges",
           "lib_path",
           "brute_trussness", "brute_h_support", "truss_components",
           "hindex_sequence", "hindex_trussness", "accounting"]
