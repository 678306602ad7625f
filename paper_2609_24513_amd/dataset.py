"""The paper's own dataset-level overlap join (Sections 3.2 and 3.5), beside
the per-pair path: one BVH over every triangle of a dataset, every unique
edge of the other dataset traced against it with all hits collected, and the
object pairs materialised by one of three strategies (Section 3.5, Fig. 5):

  "two_pass"   count the records per source group, allocate exactly, write
               them in a second tracing pass, then sort + unique;
  "estimated"  one tracing pass into a hashmap that drops duplicates on
               insert, of 2x the selectivity estimate's slots (load factor
               0.5), doubled and traced again if it fills;
  "fixed"      the same with a fixed number of slots.

Every step runs in the library's kernels (dataset_trace, pairs_unique,
estimate_pairs, dataset_tri_objects); this module marshals arguments, reads
the device counts that size the next allocation, and times the phases.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from . import MeshBlob, _dev, _stream_ptr, _torch, _ws

STRATEGIES = ("two_pass", "estimated", "fixed")
LOAD_FACTOR = 0.5


def merge_dataset(S):
    """The dataset as one mesh (faces in dataset order, vertex ids global)."""
    from .synth import MeshSet
    faces = np.asarray(S.faces, np.int64).copy()
    for m in range(S.n_meshes):
        faces[S.face_off[m]:S.face_off[m + 1]] += int(S.vert_off[m])
    return MeshSet(np.asarray(S.verts, np.float32), faces.astype(np.int32),
                   np.array([0, S.verts.shape[0]], np.int64), np.array([0, faces.shape[0]], np.int64))


def max_groups(S) -> int:
    """Upper bound of a per-mesh blob's 64-segment groups (3F/64 + M + 1)."""
    return 3 * int(S.faces.shape[0]) // 64 + int(S.n_meshes) + 1


class DatasetBlob:
    """A dataset-level blob (one BVH over all triangles) and its
    triangle-to-object map."""

    def __init__(self, blob: MeshBlob, tri_obj, n_objects: int, f_total: int):
        self.blob = blob
        self.tri_obj = tri_obj
        self.n_objects = int(n_objects)
        self.f_total = int(f_total)

    @property
    def width(self) -> int:
        return self.blob.width

    @classmethod
    def build(cls, S, width: int = 8, leaf_size: int = 2, builder: int = 0, stream=None):
        torch = _torch()
        blob = MeshBlob.build(merge_dataset(S), width=width, leaf_size=leaf_size, builder=builder, stream=stream)
        F = int(S.faces.shape[0])
        tri_obj = torch.empty(max(F, 1), dtype=torch.int32, device="cuda")
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        fo = _dev(S.face_off, torch.int64)
        _lib.check(_lib.load().dataset_tri_objects(blob.ptr, fo.data_ptr(), int(S.n_meshes), tri_obj.data_ptr(), F,
                                                   status.data_ptr(), _stream_ptr(stream)))
        torch.cuda.synchronize()
        if int(status.item()) != 0:
            raise _lib.PierceError(int(status.item()), "dataset_tri_objects: face outside every object")
        return cls(blob, tri_obj, S.n_meshes, F)


def estimate(A: MeshBlob, B: MeshBlob, cells: int = 32, stream=None) -> float:
    """Selectivity estimate of Section 3.5 (estimate_pairs), synchronised."""
    torch = _torch()
    lib = _lib.load()
    wb = ctypes.c_size_t(0)
    _lib.check(lib.estimate_pairs_ws_bytes(A.n_meshes, B.n_meshes, int(cells), ctypes.byref(wb)))
    ws = _ws(wb.value)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    _lib.check(lib.estimate_pairs(A.ptr, A.n_meshes, B.ptr, B.n_meshes, int(cells), out.data_ptr(), ws.data_ptr(),
                                  ws.numel(), _stream_ptr(stream)))
    return float(out.item())


class _Tracer:
    def __init__(self, src: MeshBlob, src_groups: int, dst: DatasetBlob, flip: int):
        torch = _torch()
        self.src, self.dst, self.flip, self.groups = src, dst, flip, int(src_groups)
        wb = ctypes.c_size_t(0)
        _lib.check(_lib.load().dataset_trace_ws_bytes(self.groups, ctypes.byref(wb)))
        self.ws = _ws(wb.value)
        self.counts = torch.zeros(self.groups + 1, dtype=torch.int64, device="cuda")
        self.n = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.stats = torch.zeros(len(_lib.DATASET_FIELDS), dtype=torch.int64, device="cuda")
        self.status = torch.zeros(1, dtype=torch.int32, device="cuda")

    def run(self, op: int, keys=None, key_cap: int = 0, stream=None):
        prm = _lib.DatasetParams(op, self.flip, self.dst.width, 0, int(key_cap))
        _lib.check(_lib.load().dataset_trace(
            self.src.ptr, self.src.n_meshes, self.dst.blob.ptr, self.dst.tri_obj.data_ptr(), self.dst.n_objects,
            ctypes.byref(prm), self.counts.data_ptr(), self.groups, None if keys is None else keys.data_ptr(),
            self.n.data_ptr(), self.stats.data_ptr(), self.status.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
            _stream_ptr(stream)))

    def stats_dict(self) -> dict:
        v = self.stats.cpu().numpy().astype(np.uint64)
        return {k: int(x) for k, x in zip(_lib.DATASET_FIELDS, v)}


def _unique(keys, n_keys: int, stream=None):
    torch = _torch()
    lib = _lib.load()
    wb = ctypes.c_size_t(0)
    _lib.check(lib.pairs_unique_ws_bytes(int(n_keys), ctypes.byref(wb)))
    ws = _ws(wb.value)
    out = torch.empty((max(int(n_keys), 1), 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    _lib.check(lib.pairs_unique(keys.data_ptr(), int(n_keys), out.data_ptr(), int(out.shape[0]), cnt.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return out, cnt


MAX_SLOTS = 1 << 30


def _pow2(n: int) -> int:
    return min(MAX_SLOTS, 1 << max(2, int(np.ceil(np.log2(max(n, 1))))))


def auto_cells(A: MeshBlob, B: MeshBlob, per_side: float = 4.0, max_cells: int = 64) -> int:
    """Grid resolution for the estimate (the paper does not fix it): cells of
    at least `per_side` mean object sides, so that most objects touch one
    cell and few share a cell only by straddling its boundary."""
    b = np.concatenate([A.boxes().cpu().numpy(), B.boxes().cpu().numpy()]).astype(np.float64)
    b = b[np.all(b[:, 3:] >= b[:, :3], axis=1)]
    if b.shape[0] == 0:
        return 1
    side = float((b[:, 3:] - b[:, :3]).mean())
    extent = float((b[:, 3:].max(axis=0) - b[:, :3].min(axis=0)).max())
    return int(min(max_cells, max(1, np.floor(extent / max(per_side * side, 1e-30)))))


def join_dataset(A: MeshBlob, B: MeshBlob, DA: DatasetBlob, DB: DatasetBlob, groups_a: int, groups_b: int,
                 strategy: str = "estimated", fixed_slots: Optional[int] = None, cells: Optional[int] = None,
                 stream=None):
    """Overlap join of datasets A and B by the dataset-level design: A's
    edges against DB and B's edges against DA.  A, B are the per-mesh blobs
    (their edges), DA, DB the dataset-level blobs, groups_a / groups_b bounds
    of the per-mesh blobs' groups (max_groups).  Returns (pairs int32[n, 2]
    sorted, info) with the phase times (ms, device events), the output
    memory allocated (bytes), relaunches and the trace statistics."""
    torch = _torch()
    if strategy not in STRATEGIES:
        raise ValueError("strategy must be one of %s" % (STRATEGIES,))
    ta, tb = _Tracer(A, groups_a, DB, 0), _Tracer(B, groups_b, DA, 1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    info = {"strategy": strategy, "relaunches": 0}
    ev[0].record()
    if strategy == "two_pass":
        ta.run(0, stream=stream)
        tb.run(0, stream=stream)
        ev[1].record()
        na, nb = int(ta.n.item()), int(tb.n.item())   # the host allocates between the passes
        keys = torch.empty(max(na + nb, 1), dtype=torch.int64, device="cuda")
        if na:
            ta.run(1, keys, na, stream=stream)
        if nb:
            tb.run(1, keys[na:], nb, stream=stream)
        n_keys = na + nb
        info["records"] = n_keys
        info["output_bytes"] = 8 * n_keys
    else:
        if strategy == "estimated":
            cells = cells or auto_cells(A, B)
            est = estimate(A, B, cells, stream=stream)
            slots = _pow2(int(np.ceil(est / LOAD_FACTOR)))
            info["estimate"] = est
            info["cells"] = cells
        else:
            slots = _pow2(int(fixed_slots or (1 << 27)))
        ev[1].record()
        while True:
            keys = torch.empty(slots, dtype=torch.int64, device="cuda")
            ta.run(3, keys, slots, stream=stream)          # clear
            ta.run(2, keys, slots, stream=stream)
            tb.run(2, keys, slots, stream=stream)
            over = int(ta.stats[6].item()) + int(tb.stats[6].item())
            if over == 0:
                break
            if slots >= MAX_SLOTS:
                raise _lib.PierceError(_lib.PR_E_CAPACITY, "more than %d distinct pairs" % MAX_SLOTS)
            slots *= 2                                      # the table filled up: twice the slots, trace again
            info["relaunches"] += 1
        n_keys = slots
        info["slots"] = slots
        info["output_bytes"] = 8 * slots
    ev[2].record()
    out, cnt = _unique(keys, n_keys, stream=stream)
    ev[3].record()
    torch.cuda.synchronize()
    for t in (ta, tb):
        if int(t.status.item()) != 0:
            raise _lib.PierceError(int(t.status.item()), "dataset_trace failed")
    n = int(cnt.item())
    info.update({"pairs": n, "ms": ev[0].elapsed_time(ev[3]), "prepare_ms": ev[0].elapsed_time(ev[1]),
                 "trace_ms": ev[1].elapsed_time(ev[2]), "unique_ms": ev[2].elapsed_time(ev[3]),
                 "stats_ab": ta.stats_dict(), "stats_ba": tb.stats_dict()})
    return out[:n].cpu().numpy(), info
