"""Seeded near-degenerate triangle pairs (test input recipe).

Each case is a pair of one-triangle meshes built so that the closed
segment-triangle tests of the refinement sit at or next to a decision
boundary: a vertex rounded onto the other triangle's plane or edge line,
shared vertices, edges crossing edges, axis-parallel edges (zero direction
components in the slab test), exactly coplanar and nearly coplanar
triangles, and large translations that leave only a few bits for the
differences.  Pairs are scaled by 2^k with k spread over [-40, 40] (exact),
and a few fall outside the range where the FP32 error bounds apply.
Non-degenerate triangles only (the exact oracle screens them).
"""
from __future__ import annotations

import numpy as np

FAMILIES = ["plane_vertex", "edge_vertex", "shared_vertex", "edge_edge", "axis_parallel", "coplanar",
            "offset_plane"]


def _rand_tri(rng, scale=1.0):
    return rng.uniform(-1.0, 1.0, size=(3, 3)) * scale


def _one(rng, fam):
    t = _rand_tri(rng)
    u = _rand_tri(rng)
    a, b, c = t
    if fam == "plane_vertex":
        s, r = rng.uniform(-0.2, 1.2, size=2)
        u[0] = a + s * (b - a) + r * (c - a)
        if rng.uniform() < 0.5:          # the rest of u on one side: touching, or not
            n = np.cross(b - a, c - a)
            side = 1.0 if rng.uniform() < 0.5 else -1.0
            u[1] = u[0] + side * n * rng.uniform(0.1, 1.0) + rng.normal(size=3) * 0.3
            u[2] = u[0] + side * n * rng.uniform(0.1, 1.0) + rng.normal(size=3) * 0.3
    elif fam == "edge_vertex":
        s = rng.uniform(-0.05, 1.05)
        u[0] = a + s * (b - a)
    elif fam == "shared_vertex":
        u[0] = t[rng.integers(0, 3)]
        if rng.uniform() < 0.3:
            u[1] = t[rng.integers(0, 3)]
    elif fam == "edge_edge":
        s = rng.uniform(-0.05, 1.05)
        m = a + s * (b - a)
        d = rng.normal(size=3)
        e = rng.uniform(1e-3, 0.5)
        u[0] = m + e * d
        u[1] = m - e * d * rng.uniform(0.5, 2.0)
    elif fam == "axis_parallel":
        # grid triangles with edges along coordinate axes; contacts exact
        k = rng.integers(1, 5)
        t = np.zeros((3, 3))
        ax = rng.permutation(3)
        t[1, ax[0]] = k
        t[2, ax[1]] = k
        t += rng.integers(-2, 3, size=3)
        u = np.zeros((3, 3))
        bx = rng.permutation(3)
        u[1, bx[0]] = rng.integers(1, 5)
        u[2, bx[1]] = rng.integers(1, 5)
        u += rng.integers(-2, 3, size=3) + rng.integers(0, 2, size=3) * 0.5
    elif fam == "coplanar":
        z = rng.uniform(-1, 1)
        t = rng.integers(-8, 9, size=(3, 3)) / 8.0
        u = rng.integers(-8, 9, size=(3, 3)) / 8.0
        ax = rng.integers(0, 3)
        t[:, ax] = z
        u[:, ax] = z
    elif fam == "offset_plane":
        # u = t moved a hair along its normal (or not at all), with a twist
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        h = rng.choice([0.0, 1e-7, -1e-7, 1e-5, 3e-8])
        u = t + h * n + rng.normal(size=(3, 3)) * rng.choice([0.0, 0.2])
        u = u[rng.permutation(3)]
    # translation far from the origin: few bits left for the differences
    if rng.uniform() < 0.15:
        off = rng.uniform(-1, 1, size=3) * 2.0 ** rng.integers(8, 20)
        t = t + off
        u = u + off
    k = int(rng.integers(-40, 41)) if rng.uniform() < 0.5 else 0
    if rng.uniform() < 0.01:
        k = int(rng.choice([-70, 60]))   # outside the FP32-bound range
    t = np.ldexp(t.astype(np.float32), k).astype(np.float32)
    u = np.ldexp(u.astype(np.float32), k).astype(np.float32)
    return t, u


def make_pairs(n, seed=77):
    """(T f32[n,3,3], U f32[n,3,3], family index int[n]) with every triangle
    non-degenerate."""
    import oracle
    rng = np.random.default_rng(seed)
    T, U, F = [], [], []
    fam_ids = rng.integers(0, len(FAMILIES), size=4 * n)
    i = 0
    while len(T) < n:
        fam = FAMILIES[fam_ids[i % fam_ids.shape[0]]]
        i += 1
        t, u = _one(rng, fam)
        if not (np.all(np.isfinite(t)) and np.all(np.isfinite(u))):
            continue
        try:
            oracle.tri_tri(t, t)
            oracle.tri_tri(u, u)
        except oracle.OracleError:
            continue
        T.append(t)
        U.append(u)
        F.append(FAMILIES.index(fam))
    return np.array(T, np.float32), np.array(U, np.float32), np.array(F)


def as_meshsets(T, U):
    """Two datasets of one-triangle meshes: A[i] = T[i], B[i] = U[i]."""
    from paper_2609_24513_amd import synth
    n = T.shape[0]
    off = np.arange(n + 1, dtype=np.int64)
    faces = np.tile(np.array([[0, 1, 2]], np.int32), (n, 1))
    A = synth.MeshSet(np.ascontiguousarray(T.reshape(-1, 3)), faces.copy(), off * 3, off.copy())
    B = synth.MeshSet(np.ascontiguousarray(U.reshape(-1, 3)), faces.copy(), off * 3, off.copy())
    return A, B
