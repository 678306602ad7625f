"""Selectivity estimate of the overlap join (Section 3.5, the Minkowski-sum
histogram that sizes the result hashmap), written out step by step in the
paper's order, in FP64.  Test infrastructure only.

Per dataset k and grid cell: N_k objects whose box touches the (closed) cell,
S_k the mean box side (width, height and depth averaged per object, then over
the objects), VolRatio_k the mean ratio of mesh volume to box volume.  Per
cell: V_int = (S_1 + S_2 + eps)^3, P_base = V_int / V_cell,
R = sqrt(VolRatio_1 VolRatio_2), F_shape = R^gamma, P = min(P_base F_shape, 1),
E = N_1 N_2 P; the estimate is the sum over cells where both datasets are
present.

Readings (the paper leaves these open): the grid spans the union of the two
datasets' boxes with `cells` cells per axis (a cube per cell is not
required: cells are boxes); a box touches every cell whose closed extent it
meets; the mesh volume is the absolute value of the divergence-theorem sum
over its triangles; a box of zero volume has ratio 1; ratios are clamped to
[0, 1].
"""
from __future__ import annotations

import numpy as np

EPS = 1e-3
GAMMA = 0.8
LOAD_FACTOR = 0.5


def mesh_volumes(S) -> np.ndarray:
    """|sum over triangles of det(a, b, c) / 6| per mesh, FP64 on the FP32 coordinates."""
    v = np.asarray(S.verts, np.float64)
    out = np.zeros(S.n_meshes)
    for m in range(S.n_meshes):
        f = np.asarray(S.faces[S.face_off[m]:S.face_off[m + 1]], np.int64) + int(S.vert_off[m])
        if f.shape[0] == 0:
            continue
        a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
        out[m] = abs(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)
    return out


def object_stats(S, boxes: np.ndarray):
    """(box f64[M, 6], mean side f64[M], volume ratio f64[M]) of each mesh."""
    b = np.asarray(boxes, np.float64)
    ext = b[:, 3:] - b[:, :3]
    side = ext.mean(axis=1)
    bvol = ext.prod(axis=1)
    vol = mesh_volumes(S)
    ratio = np.where(bvol > 0, vol / np.where(bvol > 0, bvol, 1.0), 1.0)
    return b, side, np.clip(ratio, 0.0, 1.0)


def estimate(A, B, boxes_a: np.ndarray, boxes_b: np.ndarray, cells: int = 32) -> dict:
    """E_final for datasets A and B (boxes as f32[M, 6] lo xyz, hi xyz), with
    the per-cell statistics, on a cells^3 grid over the union of both boxes."""
    ba, sa, ra = object_stats(A, boxes_a)
    bb, sb, rb = object_stats(B, boxes_b)
    both = np.concatenate([ba, bb])
    both = both[np.all(both[:, 3:] >= both[:, :3], axis=1)]
    if both.shape[0] == 0:
        both = np.zeros((1, 6))
    lo = both[:, :3].min(axis=0)
    hi = both[:, 3:].max(axis=0)
    size = np.where(hi > lo, (hi - lo) / cells, 1.0)
    v_cell = float(np.prod(size))
    G = cells

    def accumulate(boxes, side, ratio):
        n = np.zeros((G, G, G))
        s = np.zeros((G, G, G))
        r = np.zeros((G, G, G))
        for o in range(boxes.shape[0]):
            if not np.all(boxes[o, 3:] >= boxes[o, :3]):
                continue  # a mesh without faces has no box
            # cells c with lo + c size <= box_hi and lo + (c + 1) size >= box_lo
            c0 = np.clip(np.ceil((boxes[o, :3] - lo) / size - 1.0).astype(np.int64), 0, G - 1)
            c1 = np.clip(np.floor((boxes[o, 3:] - lo) / size).astype(np.int64), 0, G - 1)
            sl = tuple(slice(int(c0[k]), int(c1[k]) + 1) for k in range(3))
            n[sl] += 1.0
            s[sl] += side[o]
            r[sl] += ratio[o]
        return n, s, r

    n1, s1, r1 = accumulate(ba, sa, ra)
    n2, s2, r2 = accumulate(bb, sb, rb)
    est = 0.0
    for idx in zip(*np.nonzero((n1 > 0) & (n2 > 0))):
        N1, N2 = n1[idx], n2[idx]
        S1, S2 = s1[idx] / N1, s2[idx] / N2
        VR1, VR2 = r1[idx] / N1, r2[idx] / N2
        v_int = (S1 + S2 + EPS) ** 3
        p_base = v_int / v_cell
        f_shape = np.sqrt(VR1 * VR2) ** GAMMA
        p = min(p_base * f_shape, 1.0)
        est += N1 * N2 * p
    return {"estimate": float(est), "cells": G, "v_cell": v_cell, "grid_lo": lo, "cell_size": size,
            "slots": int(np.ceil(est / LOAD_FACTOR))}
