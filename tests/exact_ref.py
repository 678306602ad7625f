"""Independent exact reference for pinning the oracle (test helper).

A second formulation of closed triangle-triangle intersection, written in
plain Python on exact rationals: two closed triangles meet iff an edge of
one meets the other triangle (edge-face form; the core observation of
Section 3.1 extended to closed sets, including touching and coplanar
contact).  The oracle uses a different formulation (separating axes on
exact integers), so agreement between the two pins both.

Coordinates are converted with ``Fraction(float(x))``, which is exact for
FP32 inputs.  Plain ints also work (grid cases).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def exact(x):
    if isinstance(x, (int, Fraction)):
        return x
    return Fraction(float(np.float32(x)))


def pt(p):
    return tuple(exact(c) for c in p)


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def orient3d(a, b, c, d):
    """det[b-a, c-a, d-a] (exact value)."""
    return _dot(_cross(_sub(b, a), _sub(c, a)), _sub(d, a))


def _o2(a, b, c, i, j):
    return (b[i] - a[i]) * (c[j] - a[j]) - (b[j] - a[j]) * (c[i] - a[i])


def _sign(x):
    return (x > 0) - (x < 0)


def seg_tri(p, q, a, b, c) -> bool:
    """Closed segment [p,q] meets closed triangle (a,b,c)?"""
    sp = _sign(orient3d(a, b, c, p))
    sq = _sign(orient3d(a, b, c, q))
    if sp == sq and sp != 0:
        return False
    if sp == 0 and sq == 0:
        n = _cross(_sub(b, a), _sub(c, a))
        k = next(i for i in range(3) if n[i] != 0)
        i, j = [t for t in range(3) if t != k]
        s = [_sign(_o2(p, q, v, i, j)) for v in (a, b, c)]
        if all(x > 0 for x in s) or all(x < 0 for x in s):
            return False
        for x, y, z in ((a, b, c), (b, c, a), (c, a, b)):
            sz = _sign(_o2(x, y, z, i, j))
            s1 = _sign(_o2(x, y, p, i, j))
            s2 = _sign(_o2(x, y, q, i, j))
            if s1 == s2 == -sz:
                return False
        return True
    s = [_sign(orient3d(p, q, a, b)), _sign(orient3d(p, q, b, c)), _sign(orient3d(p, q, c, a))]
    return all(x >= 0 for x in s) or all(x <= 0 for x in s)


def tri_tri_edges(t, u) -> bool:
    """Edge-face form of closed triangle-triangle intersection."""
    t = [pt(v) for v in t]
    u = [pt(v) for v in u]
    for i in range(3):
        if seg_tri(t[i], t[(i + 1) % 3], u[0], u[1], u[2]):
            return True
        if seg_tri(u[i], u[(i + 1) % 3], t[0], t[1], t[2]):
            return True
    return False


def mesh_pair_edges(va, fa, vb, fb) -> bool:
    """Mesh pair intersects: any edge of one mesh meets any face of the other
    (every edge of every triangle, no dedup).  Exact; tiny meshes only."""
    VA = [pt(v) for v in va]
    VB = [pt(v) for v in vb]
    for (F1, V1, F2, V2) in ((fa, VA, fb, VB), (fb, VB, fa, VA)):
        edges = set()
        for f in F1:
            for k in range(3):
                e = (int(f[k]), int(f[(k + 1) % 3]))
                edges.add((min(e), max(e)))
        for (i, j) in edges:
            for g in F2:
                if seg_tri(V1[i], V1[j], V2[g[0]], V2[g[1]], V2[g[2]]):
                    return True
    return False
