"""Exact CPU oracle (test infrastructure only).

Loaded by the tests, the smoke check and the benchmark's CPU-baseline leg;
the product library never imports it.  See ``oracle.cpp`` for what it
computes and why it is exact.
"""
from .oracle import (build, join, tri_tri, orient3d, OracleError, set_limb_budget, default_threads,  # noqa: F401
                     winding, inside_pairs, join_predicates, PREDICATES,
                     ORACLE_E_ARG, ORACLE_E_DEGENERATE, ORACLE_E_OVERFLOW)
from .filter import mesh_boxes, candidate_pairs, unique_edges  # noqa: F401
from . import estimate  # noqa: F401
