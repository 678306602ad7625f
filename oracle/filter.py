"""Plain definitions of the candidate filter and of the unique edges
(test infrastructure only, like the rest of ``oracle/``).

These are the checkers for the device filter and for the edge sets the BVH
build stores; they share no code with the HIP library or with the input
generators.

* Mesh box: the exact box of a mesh's triangles, i.e. the coordinate-wise
  minimum and maximum over every vertex that a face of the mesh references.
  A mesh without faces has no box and is never a candidate.
* Candidate pair (the classic filter step that the paper's single traversal
  fuses with refinement, Section 1 "Challenges" and Section 3): mesh i of A
  and mesh j of B are a candidate iff their closed boxes share a point;
  with a closed query box Q, iff box_i, box_j and Q share a point.  On every
  axis that is max(lows) <= min(highs).  Touching boxes are candidates
  (closed intervals: the reading under which contact cases survive the
  filter).  Output sorted by (i, j).
* Unique edges (Section 3.1, Step I): the edges of a mesh's faces with the
  two orientations of an edge identified, i.e. the set of (min(u, v),
  max(u, v)) over the three edges (a, b), (b, c), (c, a) of every face.
"""
from __future__ import annotations

import numpy as np

__all__ = ["mesh_boxes", "candidate_pairs", "unique_edges"]


def mesh_boxes(S) -> np.ndarray:
    """f32[M, 6] = (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z) of each mesh's
    triangles; +inf lows and -inf highs for a mesh without faces."""
    M = int(S.vert_off.shape[0] - 1)
    out = np.empty((M, 6), np.float32)
    out[:, :3] = np.inf
    out[:, 3:] = -np.inf
    verts = np.asarray(S.verts, np.float32).reshape(-1, 3)
    faces = np.asarray(S.faces, np.int64).reshape(-1, 3)
    fo = np.asarray(S.face_off, np.int64)
    nf = np.diff(fo)
    if faces.shape[0] == 0:
        return out
    # every face's three vertices (global ids: the mesh's vertex offset plus
    # the face's local ids), then the minimum and maximum over a mesh's faces
    owner = np.repeat(np.arange(M), nf)
    p = verts[np.asarray(S.vert_off, np.int64)[owner][:, None] + faces]       # [F, 3 vertices, 3 coords]
    lo, hi = p.min(axis=1), p.max(axis=1)
    has = nf > 0
    out[has, :3] = np.minimum.reduceat(lo, fo[:-1][has], axis=0)
    out[has, 3:] = np.maximum.reduceat(hi, fo[:-1][has], axis=0)
    return out


def candidate_pairs(box_a: np.ndarray, box_b: np.ndarray, query=None) -> np.ndarray:
    """int64[P, 2]: every (i, j) whose closed boxes (and the closed query box,
    when given) share a point, sorted by (i, j)."""
    box_a = np.asarray(box_a, np.float32).reshape(-1, 6)
    box_b = np.asarray(box_b, np.float32).reshape(-1, 6)
    ia = np.arange(box_a.shape[0])
    ib = np.arange(box_b.shape[0])
    if query is not None:
        # a box that misses Q cannot share a point with Q and another box:
        # such rows and columns are dropped before the pairwise test
        q = np.asarray(query, np.float32).reshape(6)
        ia = ia[np.all(np.maximum(box_a[:, :3], q[:3]) <= np.minimum(box_a[:, 3:], q[3:]), axis=1)]
        ib = ib[np.all(np.maximum(box_b[:, :3], q[:3]) <= np.minimum(box_b[:, 3:], q[3:]), axis=1)]
    lo_b, hi_b = box_b[ib, :3], box_b[ib, 3:]
    if query is not None:
        lo_b = np.maximum(lo_b, q[None, :3])
        hi_b = np.minimum(hi_b, q[None, 3:])
    out = []
    rows = max(1, (1 << 22) // max(1, ib.shape[0]))
    for i0 in range(0, ia.shape[0], rows):
        a = box_a[ia[i0:i0 + rows]]
        lo = np.maximum(a[:, None, :3], lo_b[None, :, :])
        hi = np.minimum(a[:, None, 3:], hi_b[None, :, :])
        ii, jj = np.nonzero(np.all(lo <= hi, axis=2))
        out.append(np.stack([ia[ii + i0], ib[jj]], 1))
    if not out:
        return np.zeros((0, 2), np.int64)
    return np.concatenate(out).astype(np.int64)


def unique_edges(faces: np.ndarray) -> np.ndarray:
    """int64[E, 2]: the unique undirected edges (min id, max id) of one mesh's
    faces, sorted."""
    f = np.asarray(faces, np.int64).reshape(-1, 3)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0) if e.shape[0] else np.zeros((0, 2), np.int64)
