"""MI355X-native refinement of a 3D spatial join over closed triangle meshes.

Python front end of libpierce_hip.so (see include/pierce.h).  Every step of
the join runs in the library's HIP kernels; this module only marshals
arguments and uses PyTorch for device memory and streams.

    A = MeshBlob.build(meshset_a, width=4, leaf_size=4)
    B = MeshBlob.build(meshset_b, width=4, leaf_size=4)
    pairs = filter_pairs(A, B)                 # closed-box candidates, sorted
    flags, stats = refine(A, B, pairs)         # 1 iff the surfaces share a point
    result = compact(pairs, flags)             # intersecting pairs, sorted
    flags, *_ = predicate(A, B, pairs, "contains")   # A_i encloses B_j (Section 3.3)
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np

from . import _lib
from ._lib import PierceError, RefineStats, STATS_FIELDS, INSIDE_FIELDS  # noqa: F401

__all__ = ["MeshBlob", "filter_pairs", "refine", "refine_static", "compact", "gather_regions", "refine_workspace",
           "PierceError", "RefineConfig", "SCHEDULES", "small_grid", "inside", "predicate", "PREDICATES",
           "predicate_workspace"]


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev(a, dtype):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device="cuda", dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)
    return t.contiguous()


def _ws(nbytes: int):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


class MeshBlob:
    """A dataset's device-resident BVH blob (build_mesh_bvh)."""

    def __init__(self, blob, n_meshes: int, width: int, leaf_size: int, status, exps=None):
        self.blob = blob
        self.n_meshes = int(n_meshes)
        self.width = int(width)
        self.leaf_size = int(leaf_size)
        self._status = status
        self._exps = exps          # device i32[2]: coordinate bit-exponent range
        self._exp_range = None

    @property
    def ptr(self) -> int:
        return int(self.blob.data_ptr())

    @classmethod
    def build(cls, meshes, width: int = 4, leaf_size: int = 4, stream=None, check_status: bool = True,
              builder: int = 0):
        """meshes: object with verts f32[V,3], faces i32[F,3] (mesh-local ids),
        vert_off i64[M+1], face_off i64[M+1] (numpy arrays or tensors).
        builder 0: the collapse opens the largest-area child; 1: the child of
        largest area x triangle count."""
        torch = _torch()
        lib = _lib.load()
        verts = _dev(meshes.verts, torch.float32).reshape(-1, 3)
        faces = _dev(meshes.faces, torch.int32).reshape(-1, 3)
        vo = _dev(meshes.vert_off, torch.int64)
        fo = _dev(meshes.face_off, torch.int64)
        M, V, F = int(vo.numel() - 1), int(verts.shape[0]), int(faces.shape[0])
        prm = _lib.BvhParams(width, leaf_size, builder, 0)
        bb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        _lib.check(lib.build_mesh_bvh_sizes(M, F, V, ctypes.byref(prm), ctypes.byref(bb), ctypes.byref(wb)))
        blob = torch.empty(int(bb.value), dtype=torch.uint8, device="cuda")
        ws = _ws(wb.value)
        status = torch.empty(1, dtype=torch.int32, device="cuda")
        _lib.check(lib.build_mesh_bvh(verts.data_ptr(), vo.data_ptr(), faces.data_ptr(), fo.data_ptr(),
                                      M, V, F, ctypes.byref(prm), blob.data_ptr(), bb.value,
                                      ws.data_ptr(), wb.value, status.data_ptr(), _stream_ptr(stream)))
        exps = torch.empty(2, dtype=torch.int32, device="cuda")
        _lib.check(lib.blob_coord_exponents(blob.data_ptr(), exps.data_ptr(), _stream_ptr(stream)))
        out = cls(blob, M, width, leaf_size, status, exps)
        out.builder = int(builder)
        if check_status:
            st = int(status.item())
            if st != -1:
                raise PierceError(_lib.PR_E_GEOMETRY, "invalid geometry at face %d" % st)
        del ws
        return out

    def status(self) -> int:
        return int(self._status.item())

    def exp_range(self):
        """(lowest, highest) exponent of a set bit over the blob's coordinates
        (read once from the device)."""
        if self._exp_range is None:
            lo, hi = (int(x) for x in self._exps.cpu().tolist())
            self._exp_range = (lo, hi)
        return self._exp_range

    def boxes(self, stream=None):
        torch = _torch()
        out = torch.empty((self.n_meshes, 6), dtype=torch.float32, device="cuda")
        _lib.check(_lib.load().blob_mesh_boxes(self.ptr, self.n_meshes, out.data_ptr(), _stream_ptr(stream)))
        return out

    def edge_counts(self, stream=None):
        torch = _torch()
        out = torch.empty(self.n_meshes, dtype=torch.int32, device="cuda")
        _lib.check(_lib.load().blob_edge_counts(self.ptr, self.n_meshes, out.data_ptr(), _stream_ptr(stream)))
        return out


def filter_pairs(A: MeshBlob, B: MeshBlob, query_box=None, cap: Optional[int] = None, stream=None,
                 sync: bool = True):
    """Closed-box candidate pairs (i in A, j in B), sorted; int32 [P, 2] on the device.
    With sync=True: synchronises to read the count, relaunches once if `cap` was too
    small, returns the pairs.  With sync=False: returns (buffer int32[cap, 2], count
    int64[1]) on the device without synchronising; the first min(count, cap) rows are
    the pairs (the caller checks count <= cap once it reads it)."""
    torch = _torch()
    lib = _lib.load()
    wb = ctypes.c_size_t(0)
    _lib.check(lib.filter_aabb_pairs_ws_bytes(A.n_meshes, B.n_meshes, ctypes.byref(wb)))
    ws = _ws(wb.value)
    q = None if query_box is None else _dev(np.asarray(query_box, np.float32).reshape(6), torch.float32)
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")  # always written by the filter
    cap = int(cap) if cap is not None else max(1024, 4 * (A.n_meshes + B.n_meshes))
    if not sync:
        out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device="cuda")
        _lib.check(lib.filter_aabb_pairs(A.ptr, A.n_meshes, B.ptr, B.n_meshes,
                                         None if q is None else q.data_ptr(), out.data_ptr(), cap,
                                         cnt.data_ptr(), ws.data_ptr(), wb.value, _stream_ptr(stream)))
        return out[:cap], cnt
    for _ in range(2):
        out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device="cuda")
        _lib.check(lib.filter_aabb_pairs(A.ptr, A.n_meshes, B.ptr, B.n_meshes,
                                         None if q is None else q.data_ptr(), out.data_ptr(), cap,
                                         cnt.data_ptr(), ws.data_ptr(), wb.value, _stream_ptr(stream)))
        n = int(cnt.item())
        if n <= cap:
            return out[:n]
        cap = n
    raise RuntimeError("filter count changed between launches")


SCHEDULES = {"auto": 0, "wave-per-pair": 1, "wave-per-segment": 2}


class RefineConfig:
    """pr_refine_params.  schedule: 0 auto, 1 wave-per-pair, 2 wave-per-segment
    (or the names in SCHEDULES); precision: 0 FP32 + deferred FP64/exact,
    1 FP64/exact only, 2 forced deferral (test mode), 3 FP32 + in-place exact
    on small grids.  With precision 0 on two blobs whose coordinates lie on one
    small power-of-two grid (see MeshBlob.exp_range), refine() uses 3."""

    def __init__(self, persistent: int = 1, precision: int = 0, queue_cap: int = 0, grid_blocks: int = 0,
                 seg_live_max: int = 0, schedule=1, survivor_cap: int = 0, ev_begin=None,
                 ev_end=None, n_dev=None, trace_budget: int = 0, lds_stack: int = 0):
        self.n_dev = n_dev        # optional device int64[1]: number of pairs to process
        self.trace_budget = trace_budget  # 0: block work sharing; > 0: continuation pass; -1: neither
        self.ev_begin = ev_begin  # optional torch.cuda.Event recorded around the traversal kernel(s)
        self.ev_end = ev_end
        self.persistent = persistent
        self.precision = precision
        self.queue_cap = queue_cap
        self.grid_blocks = grid_blocks
        self.seg_live_max = seg_live_max  # schedule 0: per-bucket table (bytes), 0 = built-in
        self.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        self.survivor_cap = survivor_cap
        self.lds_stack = lds_stack

    def params(self, width: int) -> _lib.RefineParams:
        p = _lib.RefineParams()
        p.bvh_width = width
        p.persistent = self.persistent
        p.precision = self.precision
        p.queue_cap = self.queue_cap
        p.grid_blocks = self.grid_blocks
        p.seg_live_max = self.seg_live_max
        p.schedule = self.schedule
        p.survivor_cap = self.survivor_cap
        p.ev_begin = _event_handle(self.ev_begin)
        p.ev_end = _event_handle(self.ev_end)
        p.dev_n_pairs = None if self.n_dev is None else int(self.n_dev.data_ptr())
        p.trace_budget = self.trace_budget
        p.lds_stack = self.lds_stack
        return p


def _event_handle(ev):
    if ev is None:
        return None
    if not ev.cuda_event:          # torch creates the event lazily at its first record
        ev.record()
    return int(ev.cuda_event)


def refine_workspace(n_pairs: int, width: int, cfg: Optional[RefineConfig] = None):
    cfg = cfg or RefineConfig()
    prm = cfg.params(width)
    wb = ctypes.c_size_t(0)
    _lib.check(_lib.load().refine_workspace_bytes(int(n_pairs), ctypes.byref(prm), ctypes.byref(wb)))
    return _ws(wb.value)


def small_grid(A: MeshBlob, B: MeshBlob) -> bool:
    """True when the coordinates of both blobs lie on one power-of-two grid of
    bit span at most 14 (the condition of refinement precision 3)."""
    (la, ha), (lb, hb) = A.exp_range(), B.exp_range()
    lo, hi = min(la, lb), max(ha, hb)
    return hi >= lo and hi - lo <= 14


def _params(A: MeshBlob, B: MeshBlob, cfg: RefineConfig):
    prm = cfg.params(A.width)
    if prm.precision == 0 and small_grid(A, B):
        prm.precision = 3
    return prm


def refine(A: MeshBlob, B: MeshBlob, pairs, cfg: Optional[RefineConfig] = None, ws=None, stream=None,
           flags=None, stats=None, status=None) -> Tuple[object, object, object]:
    """Runs refine_intersects.  Returns (flags u8[P], stats u64[8], status i32[1]),
    all device tensors, without synchronising."""
    torch = _torch()
    cfg = cfg or RefineConfig()
    if A.width != B.width:
        raise ValueError("blobs built with different widths")
    pairs = _dev(pairs, torch.int32).reshape(-1, 2)
    P = int(pairs.shape[0])
    prm = _params(A, B, cfg)
    if ws is None:
        ws = refine_workspace(P, A.width, cfg)
    if flags is None:
        flags = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
    if stats is None:
        stats = torch.zeros(len(STATS_FIELDS), dtype=torch.int64, device="cuda")
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
    _lib.check(_lib.load().refine_intersects(A.ptr, A.n_meshes, B.ptr, B.n_meshes, pairs.data_ptr(), P,
                                             flags.data_ptr(), ctypes.byref(prm), stats.data_ptr(),
                                             status.data_ptr(), ws.data_ptr(), ws.numel(),
                                             _stream_ptr(stream)))
    return flags[:P], stats, status


def refine_static(A: MeshBlob, B: MeshBlob, pairs, cfg: Optional[RefineConfig] = None, stream=None,
                  flags=None, stats=None, status=None) -> Tuple[object, object, object]:
    """refine_intersects_static: as refine(), with the library's static scratch
    buffer instead of a workspace (nothing is allocated by the library).  Calls
    that overlap on one GPU race: the caller serialises them."""
    torch = _torch()
    cfg = cfg or RefineConfig()
    if A.width != B.width:
        raise ValueError("blobs built with different widths")
    pairs = _dev(pairs, torch.int32).reshape(-1, 2)
    P = int(pairs.shape[0])
    prm = _params(A, B, cfg)
    if flags is None:
        flags = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
    if stats is None:
        stats = torch.zeros(len(STATS_FIELDS), dtype=torch.int64, device="cuda")
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
    _lib.check(_lib.load().refine_intersects_static(A.ptr, A.n_meshes, B.ptr, B.n_meshes, pairs.data_ptr(), P,
                                                    flags.data_ptr(), ctypes.byref(prm), stats.data_ptr(),
                                                    status.data_ptr(), _stream_ptr(stream)))
    return flags[:P], stats, status


def stats_dict(stats) -> dict:
    vals = stats.cpu().numpy().astype(np.uint64)
    return {k: int(v) for k, v in zip(STATS_FIELDS, vals)}


def inside_stats_dict(stats) -> dict:
    vals = stats.cpu().numpy().astype(np.uint64)
    return {k: int(v) for k, v in zip(INSIDE_FIELDS, vals)}


# join predicates (Sections 3.2-3.4): code of refine_predicate / inside_pairs mode
PREDICATES = {"overlap": 0, "contains": 1, "within": 2, "intersection": 3}


def inside(A: MeshBlob, B: MeshBlob, pairs, mode=0, cross=None, ws=None, stream=None, out=None, stats=None,
           status=None) -> Tuple[object, object, object]:
    """inside_pairs: the point-in-mesh test per candidate pair.  mode 0 returns
    raw bits (bit 0 rep(B_j) inside A_i, bit 1 rep(A_i) inside B_j, bits 2 / 3
    the vertex lies on the other surface); modes 1-3 (or "contains", "within",
    "intersection") combine with `cross`, the overlap flags of refine() for
    the same pairs.  Returns (out u8[P], stats u64[8], status i32[1]), device
    tensors, without synchronising."""
    torch = _torch()
    lib = _lib.load()
    mode = PREDICATES[mode] if isinstance(mode, str) else int(mode)
    pairs = _dev(pairs, torch.int32).reshape(-1, 2)
    P = int(pairs.shape[0])
    if mode != 0:
        if cross is None:
            raise ValueError("modes 1-3 need the overlap flags")
        cross = _dev(cross, torch.uint8).reshape(-1)
    if ws is None:
        wb = ctypes.c_size_t(0)
        _lib.check(lib.inside_workspace_bytes(P, ctypes.byref(wb)))
        ws = _ws(wb.value)
    if out is None:
        out = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
    if stats is None:
        stats = torch.zeros(len(INSIDE_FIELDS), dtype=torch.int64, device="cuda")
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
    _lib.check(lib.inside_pairs(A.ptr, A.n_meshes, B.ptr, B.n_meshes, pairs.data_ptr(), P, mode,
                                None if cross is None else cross.data_ptr(), out.data_ptr(), stats.data_ptr(),
                                status.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return out[:P], stats, status


def predicate_workspace(n_pairs: int, width: int, cfg: Optional[RefineConfig] = None):
    cfg = cfg or RefineConfig()
    prm = cfg.params(width)
    wb = ctypes.c_size_t(0)
    _lib.check(_lib.load().refine_predicate_workspace_bytes(int(n_pairs), ctypes.byref(prm), ctypes.byref(wb)))
    return _ws(wb.value)


def predicate(A: MeshBlob, B: MeshBlob, pairs, pred="intersection", cfg: Optional[RefineConfig] = None, ws=None,
              stream=None, flags=None, stats=None, istats=None, status=None):
    """refine_predicate: one join predicate ("overlap", "contains", "within",
    "intersection" or 0-3) per candidate pair.  Returns (flags u8[P], refine
    stats u64[14], inside stats u64[8], status i32[1]), device tensors, without
    synchronising."""
    torch = _torch()
    cfg = cfg or RefineConfig()
    if A.width != B.width:
        raise ValueError("blobs built with different widths")
    code = PREDICATES[pred] if isinstance(pred, str) else int(pred)
    pairs = _dev(pairs, torch.int32).reshape(-1, 2)
    P = int(pairs.shape[0])
    prm = _params(A, B, cfg)
    if ws is None:
        ws = predicate_workspace(P, A.width, cfg)
    if flags is None:
        flags = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
    if stats is None:
        stats = torch.zeros(len(STATS_FIELDS), dtype=torch.int64, device="cuda")
    if istats is None:
        istats = torch.zeros(len(INSIDE_FIELDS), dtype=torch.int64, device="cuda")
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
    _lib.check(_lib.load().refine_predicate(A.ptr, A.n_meshes, B.ptr, B.n_meshes, pairs.data_ptr(), P, code,
                                            flags.data_ptr(), ctypes.byref(prm), stats.data_ptr(),
                                            istats.data_ptr(), status.data_ptr(), ws.data_ptr(), ws.numel(),
                                            _stream_ptr(stream)))
    return flags[:P], stats, istats, status


def gather_regions(regions, region_cap: int, counts, n_regions: int, out, total, stream=None):
    """gather_pair_regions: the leading pairs of n_regions regions of `region_cap`
    pairs each (counts: device int64[n_regions]) concatenated into `out` (device
    int32[cap, 2]); the length goes to `total` (device int64[1]).  No sync."""
    _lib.check(_lib.load().gather_pair_regions(regions.data_ptr(), int(region_cap), counts.data_ptr(),
                                                int(n_regions), out.data_ptr(), int(out.shape[0]),
                                                total.data_ptr(), _stream_ptr(stream)))
    return out, total


def compact(pairs, flags, stream=None, n_dev=None, sync: bool = True):
    """Pairs whose flag is 1, in input order.  n_dev: optional device int64[1], the
    number of leading pairs to consider.  sync=True synchronises to read the count and
    returns the pairs; sync=False returns (buffer int32[P, 2], count int64[1])."""
    torch = _torch()
    lib = _lib.load()
    pairs = _dev(pairs, torch.int32).reshape(-1, 2)
    P = int(pairs.shape[0])
    wb = ctypes.c_size_t(0)
    _lib.check(lib.compact_pairs_ws_bytes(P, ctypes.byref(wb)))
    ws = _ws(wb.value)
    out = torch.empty((max(P, 1), 2), dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")  # always written by the compaction
    _lib.check(lib.compact_pairs(pairs.data_ptr(), flags.data_ptr(), P,
                                 None if n_dev is None else n_dev.data_ptr(), out.data_ptr(), P,
                                 cnt.data_ptr(), ws.data_ptr(), wb.value, _stream_ptr(stream)))
    if not sync:
        return out, cnt
    return out[:int(cnt.item())]
