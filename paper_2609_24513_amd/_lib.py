"""ctypes declarations of the C ABI in include/pierce.h (argument marshalling only).

The shared library is loaded from this directory.  There is no fallback:
if libpierce_hip.so is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpierce_hip.so")

PR_OK = 0
PR_E_ARG = -1
PR_E_CAPACITY = -2
PR_E_GEOMETRY = -3
PR_E_DEVICE = -4
PR_E_UNSUPPORTED = -5
ABI_VERSION = 8

EXPORTS = [
    "pr_last_error", "pr_abi_version", "build_mesh_bvh_sizes", "build_mesh_bvh", "blob_mesh_boxes",
    "blob_edge_counts", "filter_aabb_pairs_ws_bytes", "filter_aabb_pairs", "refine_workspace_bytes",
    "refine_intersects", "compact_pairs_ws_bytes", "compact_pairs", "gather_pair_regions",
    "refine_static_scratch_bytes", "refine_intersects_static", "blob_coord_exponents", "build_mesh_bvh_bytes",
    "inside_workspace_bytes", "inside_pairs", "refine_predicate_workspace_bytes", "refine_predicate",
    "dataset_tri_objects", "dataset_trace_ws_bytes", "dataset_trace", "pairs_unique_ws_bytes", "pairs_unique",
    "estimate_pairs_ws_bytes", "estimate_pairs",
]


class PierceError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("pierce error %d: %s" % (code, msg))
        self.code = code


class BvhParams(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("builder", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class RefineParams(ctypes.Structure):
    _fields_ = [("bvh_width", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("seg_live_max", ctypes.c_uint32),
                ("schedule", ctypes.c_int32), ("survivor_cap", ctypes.c_int32),
                ("ev_begin", ctypes.c_void_p), ("ev_end", ctypes.c_void_p),
                ("dev_n_pairs", ctypes.c_void_p), ("trace_budget", ctypes.c_int32), ("lds_stack", ctypes.c_int32)]


class RefineStats(ctypes.Structure):
    _fields_ = [("segments", ctypes.c_uint64), ("node_visits", ctypes.c_uint64),
                ("tri_tests", ctypes.c_uint64), ("fp32_ambiguous", ctypes.c_uint64),
                ("fp64_filter_ambiguous", ctypes.c_uint64), ("exact_decided", ctypes.c_uint64),
                ("pairs_true", ctypes.c_uint64), ("queue_overflow", ctypes.c_uint64),
                ("groups", ctypes.c_uint64), ("tri_fetches", ctypes.c_uint64),
                ("groups_box_pass", ctypes.c_uint64), ("groups_traversed", ctypes.c_uint64),
                ("max_group_node_visits", ctypes.c_uint64), ("max_group_leaf_fetches", ctypes.c_uint64)]


STATS_FIELDS = [f for f, _ in RefineStats._fields_]


class InsideStats(ctypes.Structure):
    _fields_ = [("rays", ctypes.c_uint64), ("box_miss", ctypes.c_uint64), ("node_visits", ctypes.c_uint64),
                ("tri_tests", ctypes.c_uint64), ("crossings", ctypes.c_uint64), ("exact_signs", ctypes.c_uint64),
                ("on_surface", ctypes.c_uint64), ("deep", ctypes.c_uint64)]


INSIDE_FIELDS = [f for f, _ in InsideStats._fields_]


class DatasetParams(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("flip", ctypes.c_int32), ("width", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("key_cap", ctypes.c_int64)]


class DatasetStats(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_uint64), ("node_visits", ctypes.c_uint64), ("tri_tests", ctypes.c_uint64),
                ("hits", ctypes.c_uint64), ("records", ctypes.c_uint64), ("exact", ctypes.c_uint64),
                ("overflow", ctypes.c_uint64), ("new_keys", ctypes.c_uint64)]


DATASET_FIELDS = [f for f, _ in DatasetStats._fields_]

_lock = threading.Lock()
_lib = None

vp = ctypes.c_void_p
i64 = ctypes.c_int64
i32 = ctypes.c_int32
szp = ctypes.POINTER(ctypes.c_size_t)


def load():
    """Loads libpierce_hip.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpierce_hip.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2609_24513_amd.build_ext)")
        lib = ctypes.CDLL(LIB_PATH)
        lib.pr_last_error.restype = ctypes.c_char_p
        lib.pr_last_error.argtypes = []
        lib.pr_abi_version.restype = ctypes.c_int
        lib.build_mesh_bvh_sizes.argtypes = [i64, i64, i64, ctypes.POINTER(BvhParams), szp, szp]
        lib.build_mesh_bvh_bytes.argtypes = [i64, i64, i64, ctypes.POINTER(BvhParams)]
        lib.build_mesh_bvh.argtypes = [vp, vp, vp, vp, i64, i64, i64, ctypes.POINTER(BvhParams),
                                       vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp, vp]
        lib.blob_mesh_boxes.argtypes = [vp, i64, vp, vp]
        lib.blob_edge_counts.argtypes = [vp, i64, vp, vp]
        lib.blob_coord_exponents.argtypes = [vp, vp, vp]
        lib.filter_aabb_pairs_ws_bytes.argtypes = [i64, i64, szp]
        lib.filter_aabb_pairs.argtypes = [vp, i64, vp, i64, vp, vp, i64, vp, vp, ctypes.c_size_t, vp]
        lib.refine_workspace_bytes.argtypes = [i64, ctypes.POINTER(RefineParams), szp]
        lib.refine_intersects.argtypes = [vp, i64, vp, i64, vp, i64, vp, ctypes.POINTER(RefineParams),
                                          vp, vp, vp, ctypes.c_size_t, vp]
        lib.compact_pairs_ws_bytes.argtypes = [i64, szp]
        lib.compact_pairs.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, ctypes.c_size_t, vp]
        lib.gather_pair_regions.argtypes = [vp, i64, vp, i64, vp, i64, vp, vp]
        lib.refine_intersects_static.argtypes = [vp, i64, vp, i64, vp, i64, vp, ctypes.POINTER(RefineParams),
                                                 vp, vp, vp]
        lib.refine_static_scratch_bytes.argtypes = []
        lib.inside_workspace_bytes.argtypes = [i64, szp]
        lib.inside_pairs.argtypes = [vp, i64, vp, i64, vp, i64, i32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        lib.refine_predicate_workspace_bytes.argtypes = [i64, ctypes.POINTER(RefineParams), szp]
        lib.refine_predicate.argtypes = [vp, i64, vp, i64, vp, i64, i32, vp, ctypes.POINTER(RefineParams),
                                         vp, vp, vp, vp, ctypes.c_size_t, vp]
        lib.dataset_tri_objects.argtypes = [vp, vp, i64, vp, i64, vp, vp]
        lib.dataset_trace_ws_bytes.argtypes = [i64, szp]
        lib.dataset_trace.argtypes = [vp, i64, vp, vp, i64, ctypes.POINTER(DatasetParams), vp, i64, vp, vp, vp, vp,
                                      vp, ctypes.c_size_t, vp]
        lib.pairs_unique_ws_bytes.argtypes = [i64, szp]
        lib.pairs_unique.argtypes = [vp, i64, vp, i64, vp, vp, ctypes.c_size_t, vp]
        lib.estimate_pairs_ws_bytes.argtypes = [i64, i64, i32, szp]
        lib.estimate_pairs.argtypes = [vp, i64, vp, i64, i32, vp, vp, ctypes.c_size_t, vp]
        for name in EXPORTS[2:]:
            getattr(lib, name).restype = ctypes.c_int
        lib.refine_static_scratch_bytes.restype = ctypes.c_size_t
        lib.build_mesh_bvh_bytes.restype = ctypes.c_size_t
        if lib.pr_abi_version() != ABI_VERSION:
            raise RuntimeError("libpierce_hip.so ABI %d != %d" % (lib.pr_abi_version(), ABI_VERSION))
        _lib = lib
        return lib


def check(code: int) -> None:
    if code != PR_OK:
        msg = load().pr_last_error().decode(errors="replace")
        raise PierceError(code, msg)
