"""Seeded mesh generators for the point-in-mesh and containment tests (both
the oracle pins and the GPU parity tests use them).  Geometry only: nothing
here decides containment or intersection."""
import itertools

import numpy as np

from paper_2609_24513_amd import synth

TET_V = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
TET_F = [[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]]
OCT_V = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]
OCT_F = [[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]]
CUBE_V = [[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)]
CUBE_F = [[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
          [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]]


def mesh_set(*meshes):
    return synth.concat_meshes([(np.asarray(v, np.float64), np.asarray(f)) for v, f in meshes])


def box(lo, hi):
    """The 8 corners of [lo, hi] in CUBE_V's order (CUBE_F faces outward)."""
    return [[(lo[0], hi[0])[i], (lo[1], hi[1])[j], (lo[2], hi[2])[k]]
            for i in (0, 1) for j in (0, 1) for k in (0, 1)]


def lattice(lo, hi, step):
    ax = np.arange(lo, hi + step / 2, step)
    return [np.array(p) for p in itertools.product(ax, ax, ax)]


def probes(points, size=2.0 ** -7):
    """One small tetrahedron per point, its first face's first corner at the
    point (so the point is the mesh's representative vertex); the other
    corners lie at +size along x, y and z."""
    ms = []
    for p in points:
        p = np.asarray(p, np.float64)
        ms.append((p[None] + size * np.asarray(TET_V, np.float64), np.asarray(TET_F)))
    return synth.concat_meshes(ms)


def torus(R, r, nu, nv):
    """Torus about the z axis, (nu x nv) quads split in two, faces outward."""
    u = 2 * np.pi * np.arange(nu) / nu
    v = 2 * np.pi * np.arange(nv) / nv
    uu, vv = np.meshgrid(u, v, indexing="ij")
    verts = np.stack([(R + r * np.cos(vv)) * np.cos(uu), (R + r * np.cos(vv)) * np.sin(uu), r * np.sin(vv)],
                     -1).reshape(-1, 3)
    faces = []
    for i in range(nu):
        for j in range(nv):
            a, b = i * nv + j, ((i + 1) % nu) * nv + j
            c, d = ((i + 1) % nu) * nv + (j + 1) % nv, i * nv + (j + 1) % nv
            faces += [[a, b, c], [a, c, d]]
    return verts, np.asarray(faces)


def plates(n, h=2.0 ** -10):
    """One mesh of n disjoint thin boxes stacked along z (box k spans
    z in [2kh, (2k+1)h]); each covers the column x = y = 0, so a +z ray from
    below meets all 4n of their horizontal triangles."""
    V, F = [], []
    base = np.asarray(CUBE_F)
    for k in range(n):
        z0 = 2 * k * h
        lo = [-1 - (k % 3) / 8, -1 - (k % 5) / 8, z0]
        hi = [1 + (k % 7) / 8, 1 + (k % 2) / 8, z0 + h]
        V += box(lo, hi)
        F.append(base + 8 * k)
    return np.asarray(V, np.float64), np.concatenate(F)


def spheres(seed=41, n=250, level=2):
    """Jittered icospheres: radii 0.3..1.2, B's centre at distance 0..2.8 from
    A's (skewed towards 0), so that disjoint, crossing, A-encloses-B and
    B-encloses-A pairs all occur.  Returns (A, B, [(ca, cb, va, vb)], faces)."""
    rng = np.random.default_rng(seed)
    tv, tf = synth.icosphere(level)
    nv = tv.shape[0]
    As, Bs, info = [], [], []
    for _ in range(n):
        ra, rb = rng.uniform(0.3, 1.2, size=2)
        ca = rng.uniform(0, 4, size=3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        cb = ca + d * rng.uniform(0.0, 2.8) * rng.uniform(0, 1) ** 2
        va = (ca[None] + (ra + rng.normal(0, 0.02 * ra, size=nv))[:, None] * tv).astype(np.float32)
        vb = (cb[None] + (rb + rng.normal(0, 0.02 * rb, size=nv))[:, None] * tv).astype(np.float32)
        As.append((va, tf)); Bs.append((vb, tf)); info.append((ca, cb, va, vb))
    return synth.concat_meshes(As), synth.concat_meshes(Bs), info, tf


def nested_grid_pairs(seed=7, n=300, step=2.0 ** -6):
    """Cubes and octahedra on a 2^-6 grid, B's placed inside, across, touching
    or outside A's: pairs (k, k).  Exact dyadic coordinates make contact and
    grazing +z rays (through vertices, along edges, in face planes) common."""
    rng = np.random.default_rng(seed)
    As, Bs = [], []
    shapes = [(CUBE_V, CUBE_F, 0.5), (OCT_V, OCT_F, 0.0)]
    for _ in range(n):
        va, fa, ofa = shapes[rng.integers(2)]
        vb, fb, ofb = shapes[rng.integers(2)]
        sa = 2 * step * rng.integers(16, 33)
        sb = step * rng.integers(2, 33)
        ca = rng.integers(-64, 65, size=3) * step
        cb = ca + rng.integers(-48, 49, size=3) * step
        As.append(((np.asarray(va, np.float64) - ofa) * sa + ca, np.asarray(fa)))
        Bs.append(((np.asarray(vb, np.float64) - ofb) * sb + cb, np.asarray(fb)))
    return synth.concat_meshes(As), synth.concat_meshes(Bs)
