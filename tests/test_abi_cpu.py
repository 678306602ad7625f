"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/pierce.h, and rejects host-visible argument errors before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_2609_24513_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pierce.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpierce_hip.so is not built; run __graft_entry__.build()")
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == declared


def test_abi_version(lib):
    assert lib.pr_abi_version() == _lib.ABI_VERSION


def test_struct_sizes():
    assert ctypes.sizeof(_lib.BvhParams) == 16
    assert ctypes.sizeof(_lib.RefineParams) == 64
    assert ctypes.sizeof(_lib.RefineStats) == 112
    assert ctypes.sizeof(_lib.InsideStats) == 64
    assert ctypes.sizeof(_lib.DatasetParams) == 24
    assert ctypes.sizeof(_lib.DatasetStats) == 64


@pytest.mark.parametrize("w,l,b,r", [(3, 4, 0, 0), (4, 3, 0, 0), (4, 4, 2, 0), (4, 4, -1, 0), (4, 4, 0, 1),
                                     (16, 4, 0, 0)])
def test_bvh_params_rejected(lib, w, l, b, r):
    p = _lib.BvhParams(w, l, b, r)
    bb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.build_mesh_bvh_sizes(1, 4, 4, ctypes.byref(p), ctypes.byref(bb), ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.pr_last_error().decode()


def test_bvh_sizes_rejected(lib):
    p = _lib.BvhParams(4, 4, 0, 0)
    bb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.build_mesh_bvh_sizes(-1, 4, 4, ctypes.byref(p), ctypes.byref(bb), ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.build_mesh_bvh_sizes(1, 1 << 28, 4, ctypes.byref(p), ctypes.byref(bb),
                                    ctypes.byref(wb)) == _lib.PR_E_UNSUPPORTED
    assert lib.build_mesh_bvh_sizes(1, 4, 4, None, ctypes.byref(bb), ctypes.byref(wb)) == _lib.PR_E_ARG


def test_blob_bytes_bound(lib):
    """build_mesh_bvh_bytes equals the blob bound of build_mesh_bvh_sizes and is
    0 for rejected arguments."""
    for w, l in ((2, 1), (4, 4), (8, 8)):
        p = _lib.BvhParams(w, l, 0, 0)
        n = lib.build_mesh_bvh_bytes(10, 5000, 2600, ctypes.byref(p))
        assert n > 5000 * 36 + 7500 * 24
        assert lib.build_mesh_bvh_bytes(10, 10000, 5200, ctypes.byref(p)) > n
        bb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        # the workspace query needs the HIP runtime; where it answers, the bounds agree
        if lib.build_mesh_bvh_sizes(10, 5000, 2600, ctypes.byref(p), ctypes.byref(bb), ctypes.byref(wb)) == 0:
            assert bb.value == n
    bad = _lib.BvhParams(3, 4, 0, 0)
    assert lib.build_mesh_bvh_bytes(10, 5000, 2600, ctypes.byref(bad)) == 0
    # both builders (greedy largest-area / area x triangle-count collapse) are accepted
    assert lib.build_mesh_bvh_bytes(10, 5000, 2600, ctypes.byref(_lib.BvhParams(4, 4, 1, 0))) == \
        lib.build_mesh_bvh_bytes(10, 5000, 2600, ctypes.byref(_lib.BvhParams(4, 4, 0, 0)))
    assert lib.build_mesh_bvh_bytes(-1, 5000, 2600, ctypes.byref(_lib.BvhParams(4, 4, 0, 0))) == 0


def test_build_null_pointers_rejected(lib):
    p = _lib.BvhParams(4, 4, 0, 0)
    assert lib.build_mesh_bvh(None, None, None, None, 1, 3, 1, ctypes.byref(p), None, 0, None, 0, None,
                              None) == _lib.PR_E_ARG


def _refine_params(**kw):
    p = _lib.RefineParams()
    p.bvh_width = kw.get("w", 4)
    p.persistent = kw.get("persistent", 1)
    p.precision = kw.get("precision", 0)
    p.queue_cap = kw.get("queue_cap", 0)
    p.grid_blocks = kw.get("grid_blocks", 0)
    p.seg_live_max = kw.get("seg_live_max", 0)
    p.schedule = kw.get("schedule", 0)
    p.trace_budget = kw.get("trace_budget", 0)
    p.lds_stack = kw.get("lds_stack", 0)
    return p


@pytest.mark.parametrize("kw", [dict(w=3), dict(precision=4), dict(precision=-1), dict(persistent=2),
                                dict(queue_cap=-1), dict(grid_blocks=-5), dict(schedule=3), dict(schedule=-1),
                                dict(trace_budget=-2), dict(lds_stack=2), dict(lds_stack=-1)])
def test_refine_params_rejected(lib, kw):
    p = _refine_params(**kw)
    wb = ctypes.c_size_t(0)
    assert lib.refine_workspace_bytes(10, ctypes.byref(p), ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.refine_intersects(None, 1, None, 1, None, 10, None, ctypes.byref(p), None, None, None, 0,
                                 None) == _lib.PR_E_ARG


@pytest.mark.parametrize("kw", [dict(schedule=0), dict(schedule=1), dict(schedule=2), dict(precision=3),
                                dict(lds_stack=1), dict(seg_live_max=0x10203040)])
def test_refine_params_accepted(lib, kw):
    """Every schedule (auto, wave-per-pair, wave-per-segment), precision 3,
    the LDS stack and a per-bucket table are valid parameters."""
    p = _refine_params(**kw)
    wb = ctypes.c_size_t(0)
    assert lib.refine_workspace_bytes(10, ctypes.byref(p), ctypes.byref(wb)) == _lib.PR_OK
    assert wb.value > 0


def test_refine_reserved_and_sizes_rejected(lib):
    p = _refine_params()
    p.survivor_cap = -1
    wb = ctypes.c_size_t(0)
    assert lib.refine_workspace_bytes(10, ctypes.byref(p), ctypes.byref(wb)) == _lib.PR_E_ARG
    p = _refine_params()
    assert lib.refine_workspace_bytes(-1, ctypes.byref(p), ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.refine_workspace_bytes(1 << 30, ctypes.byref(p), ctypes.byref(wb)) == _lib.PR_E_UNSUPPORTED
    # null blobs
    assert lib.refine_intersects(None, 1, None, 1, None, 0, None, ctypes.byref(p), None, None, None, 0,
                                 None) == _lib.PR_E_ARG


def test_filter_compact_and_gather_args_rejected(lib):
    wb = ctypes.c_size_t(0)
    assert lib.filter_aabb_pairs_ws_bytes(-1, 2, ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.filter_aabb_pairs(None, 1, None, 1, None, None, 0, None, None, 0, None) == _lib.PR_E_ARG
    assert lib.compact_pairs_ws_bytes(-2, ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.compact_pairs(None, None, 5, None, None, 0, None, None, 0, None) == _lib.PR_E_ARG
    assert lib.blob_mesh_boxes(None, 3, None, None) == _lib.PR_E_ARG
    assert lib.blob_edge_counts(None, 3, None, None) == _lib.PR_E_ARG
    assert lib.blob_coord_exponents(None, None, None) == _lib.PR_E_ARG
    # gather: null total, negative sizes, null inputs with regions, too many regions
    assert lib.gather_pair_regions(None, 4, None, 0, None, 0, None, None) == _lib.PR_E_ARG
    dummy = ctypes.c_int64(0)
    assert lib.gather_pair_regions(None, -1, None, 0, None, 0, ctypes.byref(dummy), None) == _lib.PR_E_ARG
    assert lib.gather_pair_regions(None, 4, None, 2, None, 0, ctypes.byref(dummy), None) == _lib.PR_E_ARG
    assert lib.gather_pair_regions(None, 4, None, 0, None, 5, ctypes.byref(dummy), None) == _lib.PR_E_ARG
    assert lib.gather_pair_regions(ctypes.byref(dummy), 4, ctypes.byref(dummy), (1 << 20) + 1, None, 0,
                                   ctypes.byref(dummy), None) == _lib.PR_E_UNSUPPORTED


def test_inside_and_predicate_args_rejected(lib):
    """Host-visible errors of the containment entry points, before any device
    work: negative sizes, null pointers, unknown modes and predicates, a mode
    that needs overlap flags without them, a too-small workspace."""
    wb = ctypes.c_size_t(0)
    assert lib.inside_workspace_bytes(-1, ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.inside_workspace_bytes(10, None) == _lib.PR_E_ARG
    assert lib.inside_workspace_bytes(1 << 31, ctypes.byref(wb)) == _lib.PR_E_UNSUPPORTED
    assert lib.inside_workspace_bytes(1000, ctypes.byref(wb)) == _lib.PR_OK and wb.value >= 2 * 1000 * 5
    d = ctypes.c_int64(0)
    buf = ctypes.byref(d)
    # null blobs, null pairs / out with pairs, negative counts
    assert lib.inside_pairs(None, 1, buf, 1, buf, 1, 0, None, buf, None, None, buf, 1 << 20, None) == _lib.PR_E_ARG
    assert lib.inside_pairs(buf, 1, buf, 1, None, 1, 0, None, buf, None, None, buf, 1 << 20, None) == _lib.PR_E_ARG
    assert lib.inside_pairs(buf, -1, buf, 1, buf, 1, 0, None, buf, None, None, buf, 1 << 20, None) == _lib.PR_E_ARG
    for mode in (-1, 4):
        assert lib.inside_pairs(buf, 1, buf, 1, buf, 1, mode, buf, buf, None, None, buf, 1 << 20,
                                None) == _lib.PR_E_ARG
    assert lib.inside_pairs(buf, 1, buf, 1, buf, 1, 1, None, buf, None, None, buf, 1 << 20, None) == _lib.PR_E_ARG
    assert lib.inside_pairs(buf, 1, buf, 1, buf, 1, 0, None, buf, None, None, buf, 64, None) == _lib.PR_E_CAPACITY
    p = _refine_params()
    assert lib.refine_predicate_workspace_bytes(10, ctypes.byref(p), ctypes.byref(wb)) == _lib.PR_OK
    need = wb.value
    rw, iw = ctypes.c_size_t(0), ctypes.c_size_t(0)
    lib.refine_workspace_bytes(10, ctypes.byref(p), ctypes.byref(rw))
    lib.inside_workspace_bytes(10, ctypes.byref(iw))
    assert need == max(rw.value, iw.value)
    for pred in (-1, 4):
        assert lib.refine_predicate(buf, 1, buf, 1, buf, 1, pred, buf, ctypes.byref(p), None, None, None, buf,
                                    need, None) == _lib.PR_E_ARG
    assert lib.refine_predicate(buf, 1, buf, 1, buf, 1, 1, buf, ctypes.byref(p), None, None, None, buf, 64,
                                None) == _lib.PR_E_CAPACITY
    bad = _refine_params(w=3)
    assert lib.refine_predicate(buf, 1, buf, 1, buf, 1, 1, buf, ctypes.byref(bad), None, None, None, buf, need,
                                None) == _lib.PR_E_ARG


def test_dataset_args_rejected(lib):
    """Host-visible errors of the dataset-level entry points."""
    wb = ctypes.c_size_t(0)
    d = ctypes.c_int64(0)
    buf = ctypes.byref(d)
    assert lib.dataset_trace_ws_bytes(-1, ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.dataset_trace_ws_bytes(1000, ctypes.byref(wb)) == _lib.PR_OK and wb.value > 8000
    assert lib.pairs_unique_ws_bytes(-1, ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.estimate_pairs_ws_bytes(1, 1, 0, ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.estimate_pairs_ws_bytes(1, 1, 257, ctypes.byref(wb)) == _lib.PR_E_ARG
    assert lib.dataset_tri_objects(None, buf, 1, buf, 1, buf, None) == _lib.PR_E_ARG
    assert lib.dataset_tri_objects(buf, buf, 0, buf, 1, buf, None) == _lib.PR_E_ARG
    lib.dataset_trace_ws_bytes(10, ctypes.byref(wb))
    need = wb.value
    for op, flip, width, cap in ((4, 0, 4, 16), (-1, 0, 4, 16), (0, 2, 4, 16), (0, 0, 3, 16), (2, 0, 4, 12),
                                 (2, 0, 4, 0)):
        p = _lib.DatasetParams(op, flip, width, 0, cap)
        assert lib.dataset_trace(buf, 1, buf, buf, 1, ctypes.byref(p), buf, 10, buf, buf, None, buf, buf, need,
                                 None) == _lib.PR_E_ARG, (op, flip, width, cap)
    p = _lib.DatasetParams(0, 0, 4, 0, 0)
    assert lib.dataset_trace(buf, 1, buf, buf, 1, ctypes.byref(p), buf, 10, buf, buf, None, buf, buf, 64,
                             None) == _lib.PR_E_CAPACITY
    assert lib.pairs_unique(None, 5, buf, 5, buf, buf, 1 << 20, None) == _lib.PR_E_ARG
    assert lib.estimate_pairs(None, 1, buf, 1, 8, buf, buf, 1 << 20, None) == _lib.PR_E_ARG


def test_product_path_has_no_oracle_dependency():
    """The package must not import, load or call the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2609_24513_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "_oracle.so" not in txt and "oracle.cpp" not in txt, f
