"""Seeded synthetic mesh datasets.

This module only draws inputs: closed triangle meshes (flat FP32 vertex
array, mesh-local int32 face array, CSR offsets) and candidate pair lists.
It holds none of the join arithmetic, so both the exact CPU oracle and the
HIP library consume exactly the same bytes.

Geometry is computed in FP64 and rounded once to FP32 (round to nearest
even).  The random source is ``numpy.random.Generator(PCG64(seed))``.

The workload shapes stand in for the paper's datasets (Section 4.2 and
Table 1: Tissue nuclei and vessels, synthetic spheres), which are not
available here: only their shapes are imitated.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "MeshSet", "icosphere", "geodesic_sphere", "capped_tube",
    "make_c1", "make_c2", "make_c3", "make_c4", "make_c5_pool", "c5_queries",
    "concat_meshes", "uv_sphere", "SWEEP_RINGS", "make_sweep", "make_cubes",
]


@dataclasses.dataclass
class MeshSet:
    """A dataset of closed triangle meshes in flat CSR form.

    verts    f32[V_tot, 3]
    faces    i32[F_tot, 3]   vertex ids local to their mesh
    vert_off i64[M + 1]      mesh m owns verts[vert_off[m]:vert_off[m+1]]
    face_off i64[M + 1]      mesh m owns faces[face_off[m]:face_off[m+1]]
    """
    verts: np.ndarray
    faces: np.ndarray
    vert_off: np.ndarray
    face_off: np.ndarray

    @property
    def n_meshes(self) -> int:
        return int(self.vert_off.shape[0] - 1)

    def mesh(self, m: int) -> Tuple[np.ndarray, np.ndarray]:
        v = self.verts[self.vert_off[m]:self.vert_off[m + 1]]
        f = self.faces[self.face_off[m]:self.face_off[m + 1]]
        return v, f

    def aabbs(self) -> np.ndarray:
        """Exact per-mesh boxes f32[M, 6] = (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z)
        over each mesh's vertex range (every generator here references all of
        its vertices, so this is the box of the mesh's triangles)."""
        M = self.n_meshes
        lo = np.full((M, 3), np.inf, np.float32)
        hi = np.full((M, 3), -np.inf, np.float32)
        nonempty = (np.diff(self.vert_off) > 0) & (np.diff(self.face_off) > 0)
        if nonempty.any():
            idx = self.vert_off[:-1][nonempty]
            lo[nonempty] = np.minimum.reduceat(self.verts, idx, axis=0)
            hi[nonempty] = np.maximum.reduceat(self.verts, idx, axis=0)
        return np.concatenate([lo, hi], axis=1)

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.verts, self.faces, self.vert_off, self.face_off):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def subset(self, ids: Sequence[int]) -> "MeshSet":
        return concat_meshes([self.mesh(int(i)) for i in ids])


def concat_meshes(meshes: Sequence[Tuple[np.ndarray, np.ndarray]]) -> MeshSet:
    vs = [np.asarray(v, np.float32).reshape(-1, 3) for v, _ in meshes]
    fs = [np.asarray(f, np.int32).reshape(-1, 3) for _, f in meshes]
    vo = np.zeros(len(meshes) + 1, np.int64)
    fo = np.zeros(len(meshes) + 1, np.int64)
    vo[1:] = np.cumsum([v.shape[0] for v in vs])
    fo[1:] = np.cumsum([f.shape[0] for f in fs])
    verts = np.concatenate(vs) if vs else np.zeros((0, 3), np.float32)
    faces = np.concatenate(fs) if fs else np.zeros((0, 3), np.int32)
    return MeshSet(np.ascontiguousarray(verts), np.ascontiguousarray(faces), vo, fo)


# ---------------------------------------------------------------------------
# Template surfaces (unit size, FP64)
# ---------------------------------------------------------------------------

def _icosahedron() -> Tuple[np.ndarray, np.ndarray]:
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


_ICO_CACHE = {}


def icosphere(level: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit icosphere: icosahedron, `level` midpoint subdivisions, projected.

    level 2 -> V=162, F=320;  level 4 -> V=2562, F=5120.  Faces point outward.
    """
    if level in _ICO_CACHE:
        v, f = _ICO_CACHE[level]
        return v.copy(), f.copy()
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    faces = [tuple(x) for x in f]
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                a = np.asarray(verts[i]); b = np.asarray(verts[j])
                m = (a + b) / 2.0
                m /= np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    out = (np.array(verts, np.float64), np.array(faces, np.int64))
    _ICO_CACHE[level] = out
    return out[0].copy(), out[1].copy()


_GEO_CACHE = {}


def geodesic_sphere(nu: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit geodesic sphere of frequency nu: each icosahedron face is cut into
    nu^2 triangles on a barycentric grid, then projected.  V=10nu^2+2, F=20nu^2.
    Grid points shared by neighbouring faces are merged by exact equality of
    their (pre-projection) coordinates, which are computed identically."""
    if nu in _GEO_CACHE:
        v, f = _GEO_CACHE[nu]
        return v.copy(), f.copy()
    iv, ifc = _icosahedron()
    ii, jj = [], []
    for i in range(nu + 1):
        for j in range(nu + 1 - i):
            ii.append(i); jj.append(j)
    ii = np.array(ii); jj = np.array(jj); kk = nu - ii - jj
    local = -np.ones((nu + 1, nu + 1), np.int64)
    local[ii, jj] = np.arange(ii.shape[0])
    tri = []
    for i in range(nu):
        for j in range(nu - i):
            tri.append((local[i, j], local[i + 1, j], local[i, j + 1]))
            if i + j < nu - 1:
                tri.append((local[i + 1, j], local[i + 1, j + 1], local[i, j + 1]))
    tri = np.array(tri, np.int64)
    npts = ii.shape[0]
    pts = []
    for a, b, c in ifc:
        pts.append(kk[:, None] * iv[a][None] + ii[:, None] * iv[b][None] + jj[:, None] * iv[c][None])
    pts = np.concatenate(pts) / nu
    uniq, inv = np.unique(pts, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    faces = np.concatenate([inv[f * npts + tri] for f in range(ifc.shape[0])])
    verts = uniq / np.linalg.norm(uniq, axis=1, keepdims=True)
    out = (verts, faces.astype(np.int64))
    _GEO_CACHE[nu] = out
    return out[0].copy(), out[1].copy()


def _bezier(ctrl: np.ndarray, t: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Cubic Bezier points and unit tangents at parameters t."""
    p0, p1, p2, p3 = ctrl
    s = 1.0 - t
    pts = (s ** 3)[:, None] * p0 + (3 * s * s * t)[:, None] * p1 \
        + (3 * s * t * t)[:, None] * p2 + (t ** 3)[:, None] * p3
    der = (3 * s * s)[:, None] * (p1 - p0) + (6 * s * t)[:, None] * (p2 - p1) \
        + (3 * t * t)[:, None] * (p3 - p2)
    nrm = np.linalg.norm(der, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return pts, der / nrm


def capped_tube(ctrl: np.ndarray, radius: float, rings: int = 64,
                sides: int = 32) -> Tuple[np.ndarray, np.ndarray]:
    """Closed tube swept along a cubic Bezier with rotation-minimising frames
    (double reflection method of Wang, Juettler, Zheng and Liu, 2008) and
    fan caps to two centre vertices.  V = rings*sides + 2,
    F = 2*sides*(rings-1) + 2*sides; faces point outward."""
    t = np.linspace(0.0, 1.0, rings)
    pts, tan = _bezier(np.asarray(ctrl, np.float64), t)
    # initial normal: any unit vector orthogonal to the first tangent
    a = np.array([1.0, 0.0, 0.0]) if abs(tan[0, 0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    r = a - tan[0] * (a @ tan[0])
    r /= np.linalg.norm(r)
    frames = [r]
    for i in range(rings - 1):
        v1 = pts[i + 1] - pts[i]
        c1 = v1 @ v1
        if c1 == 0:
            frames.append(frames[-1]); continue
        rl = frames[-1] - (2.0 / c1) * (v1 @ frames[-1]) * v1
        tl = tan[i] - (2.0 / c1) * (v1 @ tan[i]) * v1
        v2 = tan[i + 1] - tl
        c2 = v2 @ v2
        rn = rl if c2 == 0 else rl - (2.0 / c2) * (v2 @ rl) * v2
        rn = rn - tan[i + 1] * (rn @ tan[i + 1])
        frames.append(rn / np.linalg.norm(rn))
    R = np.array(frames)
    B = np.cross(tan, R)
    ang = 2.0 * np.pi * np.arange(sides) / sides
    ring = (np.cos(ang)[None, :, None] * R[:, None, :]
            + np.sin(ang)[None, :, None] * B[:, None, :])
    verts = (pts[:, None, :] + radius * ring).reshape(-1, 3)
    c0 = rings * sides
    verts = np.concatenate([verts, pts[:1], pts[-1:]])
    return verts, _tube_faces(rings, sides)


_TUBE_CACHE = {}


def _tube_faces(rings: int, sides: int) -> np.ndarray:
    key = (rings, sides)
    if key not in _TUBE_CACHE:
        i = np.arange(rings - 1)[:, None]
        j = np.arange(sides)[None, :]
        a0 = i * sides + j
        a1 = i * sides + (j + 1) % sides
        b0 = a0 + sides
        b1 = a1 + sides
        side_f = np.stack([np.stack([a0, a1, b1], -1), np.stack([a0, b1, b0], -1)], 2).reshape(-1, 3)
        c0 = rings * sides
        last = (rings - 1) * sides
        jj = np.arange(sides)
        cap0 = np.stack([np.full(sides, c0), (jj + 1) % sides, jj], 1)
        cap1 = np.stack([np.full(sides, c0 + 1), last + jj, last + (jj + 1) % sides], 1)
        _TUBE_CACHE[key] = np.concatenate([side_f, cap0, cap1]).astype(np.int64)
    return _TUBE_CACHE[key].copy()


def _f32(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def _jittered_sphere(rng, tmpl_v, centre, r, sigma_rel):
    u = tmpl_v
    rad = r + rng.normal(0.0, sigma_rel * r, size=u.shape[0])
    return centre[None, :] + rad[:, None] * u


def make_c1(seed: int = 1, n: int = 8) -> Tuple[MeshSet, MeshSet]:
    """Tiny config: two datasets of `n` level-2 icospheres (V=162, F=320),
    r~U[0.8,1.2], centre~U[0,4]^3, per-vertex radial jitter N(0, 0.02 r)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tv, tf = icosphere(2)
    out = []
    for _ in range(2):
        meshes = []
        for _ in range(n):
            r = rng.uniform(0.8, 1.2)
            c = rng.uniform(0.0, 4.0, size=3)
            meshes.append((_f32(_jittered_sphere(rng, tv, c, r, 0.02)), tf))
        out.append(concat_meshes(meshes))
    return out[0], out[1]


def _noise_radius(rng, u: np.ndarray, amp: float, waves: int = 8) -> np.ndarray:
    """Low-frequency displacement field on unit directions u, in [-amp, amp]:
    a sum of `waves` plane waves sin(2 pi f k.u + phi), f in {1,2}, scaled so
    that its largest magnitude over the vertices is exactly 1."""
    k = rng.normal(size=(waves, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    fr = rng.integers(1, 3, size=waves).astype(np.float64)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=waves)
    n = np.sin(2.0 * np.pi * fr[None, :] * (u @ k.T) + ph[None, :]).sum(1)
    m = np.abs(n).max()
    return amp * (n / m if m > 0 else n)


def make_c2(seed: int = 2, n_nuclei: int = 10_000, n_vessels: int = 1_000,
            box: float = 1000.0, nucleus_level: int = 4) -> Tuple[MeshSet, MeshSet]:
    """Pathology-shaped config: nuclei (level-4 icospheres, r~U[3,8], radius
    r(1 + 0.15 n(u)) with low-frequency noise n in [-1,1]) and vessels
    (capped tubes of 64 rings x 32 sides along random cubic Beziers,
    P0~U[0,box]^3, P_{k+1} = P_k + U[-100,100]^3, tube radius U[2,6])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tv, tf = icosphere(nucleus_level)
    nv, nf = tv.shape[0], tf.shape[0]
    r = rng.uniform(3.0, 8.0, size=n_nuclei)
    c = rng.uniform(0.0, box, size=(n_nuclei, 3))
    waves = 8
    k = rng.normal(size=(n_nuclei, waves, 3))
    k /= np.linalg.norm(k, axis=2, keepdims=True)
    fr = rng.integers(1, 3, size=(n_nuclei, waves)).astype(np.float64)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(n_nuclei, waves))
    verts = np.empty((n_nuclei, nv, 3), np.float32)
    step = 256
    for s0 in range(0, n_nuclei, step):
        s1 = min(n_nuclei, s0 + step)
        proj = np.einsum("vd,mwd->mvw", tv, k[s0:s1])               # (m, V, waves)
        n = np.sin(2.0 * np.pi * fr[s0:s1, None, :] * proj + ph[s0:s1, None, :]).sum(2)
        n /= np.abs(n).max(axis=1, keepdims=True)
        rad = r[s0:s1, None] * (1.0 + 0.15 * n)
        verts[s0:s1] = (c[s0:s1, None, :] + rad[:, :, None] * tv[None]).astype(np.float32)
    nuc = MeshSet(verts.reshape(-1, 3), np.ascontiguousarray(np.tile(tf.astype(np.int32), (n_nuclei, 1))),
                  np.arange(n_nuclei + 1, dtype=np.int64) * nv, np.arange(n_nuclei + 1, dtype=np.int64) * nf)
    ves = []
    for _ in range(n_vessels):
        p0 = rng.uniform(0.0, box, size=3)
        steps = rng.uniform(-100.0, 100.0, size=(3, 3))
        ctrl = np.concatenate([p0[None], p0[None] + np.cumsum(steps, axis=0)])
        rho = rng.uniform(2.0, 6.0)
        v, f = capped_tube(ctrl, rho, 64, 32)
        ves.append((_f32(v), f))
    return nuc, concat_meshes(ves)


def _log_uniform_int(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def make_c3_pool(seed: int = 3, n_pool: int = 4096, f_lo: float = 500.0,
                 f_hi: float = 100_000.0) -> Tuple[MeshSet, MeshSet, np.ndarray]:
    """Batching pool: n_pool/2 noise-displaced geodesic spheres (F=20 nu^2) and
    n_pool/2 capped tubes (F = 2*sides*rings), with target face counts
    log-uniform on [f_lo, f_hi].  Returns the two halves (A: even ids,
    B: odd ids) unplaced (centred at the origin) and the realised face counts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    targets = _log_uniform_int(rng, f_lo, f_hi, n_pool)
    meshes = []
    for i, ft in enumerate(targets):
        if i % 2 == 0:
            nu = max(2, int(round(math.sqrt(ft / 20.0))))
            tv, tf = geodesic_sphere(nu)
            r = rng.uniform(3.0, 8.0)
            rad = r * (1.0 + _noise_radius(rng, tv, 0.15))
            meshes.append((rad[:, None] * tv, tf))
        else:
            sides = max(4, int(round(math.sqrt(ft / 4.0))))
            rings = max(2, int(round(ft / (2.0 * sides))))
            steps = rng.uniform(-40.0, 40.0, size=(3, 3))
            ctrl = np.concatenate([np.zeros((1, 3)), np.cumsum(steps, axis=0)])
            ctrl -= ctrl.mean(0)
            rho = rng.uniform(2.0, 6.0)
            meshes.append(capped_tube(ctrl, rho, rings, sides))
    fcount = np.array([f.shape[0] for _, f in meshes], np.int64)
    return meshes, fcount, rng


def make_c3(seed: int = 3, n_pairs: int = 50_000, n_pool: int = 4096,
            f_lo: float = 500.0, f_hi: float = 100_000.0):
    """Batching config: the pool split into halves A and B (by index parity),
    placed uniformly in a cube whose side is halved until the closed-AABB
    filter yields at least n_pairs A x B candidates; the first n_pairs in a
    seeded shuffled order are kept, sorted by (i, j).  Returns (A, B, pairs)."""
    meshes, fcount, rng = make_c3_pool(seed, n_pool, f_lo, f_hi)
    unit_c = rng.uniform(0.0, 1.0, size=(len(meshes), 3))
    lo = np.array([v.min(0) for v, _ in meshes])
    hi = np.array([v.max(0) for v, _ in meshes])
    side = 4096.0
    while True:
        off = side * unit_c
        # fl(x + o) is monotone in x, so the placed FP32 box is the rounded placed box
        box = np.concatenate([lo + off, hi + off], axis=1).astype(np.float32)
        cand = _overlap_pairs(box[0::2], box[1::2])
        if cand.shape[0] >= n_pairs or side < 1.0:
            break
        side /= 2.0
    placed = [(_f32(v + off[i][None, :]), f) for i, (v, f) in enumerate(meshes)]
    A = concat_meshes(placed[0::2]); B = concat_meshes(placed[1::2])
    order = rng.permutation(cand.shape[0])[:n_pairs]
    pairs = cand[np.sort(order)]
    return A, B, np.ascontiguousarray(pairs.astype(np.int32))


def _overlap_pairs(box_a: np.ndarray, box_b: np.ndarray) -> np.ndarray:
    """Pairs of closed boxes that overlap, sorted (i, j): used only to place
    the batching workload (the cube is shrunk until enough pairs overlap).
    The device filter is checked against the oracle's own definition."""
    out = []
    for i in range(box_a.shape[0]):
        a = box_a[i]
        ok = np.all(box_b[:, :3] <= a[3:][None, :], axis=1) & \
            np.all(box_b[:, 3:] >= a[:3][None, :], axis=1)
        js = np.nonzero(ok)[0]
        out.append(np.stack([np.full(js.shape, i), js], 1))
    return np.concatenate(out).astype(np.int64) if out else np.zeros((0, 2), np.int64)


def _snap(x: np.ndarray, step: float) -> np.ndarray:
    return np.round(np.asarray(x, np.float64) / step) * step


def make_c4(seed: int = 4, n_pairs: int = 2000, grid_bits: int = 10):
    """Precision-stress config: n_pairs (A_i, B_i) of level-4 icospheres,
    r~U[0.8,1.2], vertices snapped to a 2^-grid_bits grid, A centred at 0.
    Placement classes (intents only; the oracle decides the truth):
      30% tangent   - B's extreme vertex along -axis put on A's extreme vertex along +axis
      20% coplanar  - B = 2m - A, m = a/4 + b/2 + c/4 inside a face (a,b,c) of A
      10% on-surface- B's extreme vertex along -n_f put on (2a+b+c)/4 of a face of A
      40% random    - centre offset |d|~U[0, rA+rB+0.2] along a random direction
    Returns (A, B, pairs = (i, i), classes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tv, tf = icosphere(4)
    step = 2.0 ** -grid_bits
    cls_names = ["tangent", "coplanar", "on_surface", "random"]
    cum = np.cumsum([0.3, 0.2, 0.1, 0.4])
    A_list, B_list, classes = [], [], []
    for _ in range(n_pairs):
        u = rng.uniform()
        cls = int(np.searchsorted(cum, u, side="right"))
        cls = min(cls, 3)
        ra, rb = rng.uniform(0.8, 1.2, size=2)
        va = _snap(ra * tv, step)
        vb0 = _snap(rb * tv, step)
        if cls == 0:
            ax = int(rng.integers(0, 3)); sgn = 1.0 if rng.uniform() < 0.5 else -1.0
            ia = int(np.argmax(sgn * va[:, ax]))
            ib = int(np.argmin(sgn * vb0[:, ax]))
            vb = vb0 + (va[ia] - vb0[ib])[None, :]
        elif cls == 1:
            fi = int(rng.integers(0, tf.shape[0]))
            a, b, c = va[tf[fi]]
            m = a / 4 + b / 2 + c / 4
            vb = 2.0 * m[None, :] - va
        elif cls == 2:
            fi = int(rng.integers(0, tf.shape[0]))
            a, b, c = va[tf[fi]]
            n = np.cross(b - a, c - a)
            ib = int(np.argmax(-(vb0 @ n)))
            tgt = (2 * a + b + c) / 4
            vb = vb0 + (tgt - vb0[ib])[None, :]
        else:
            d = rng.normal(size=3); d /= np.linalg.norm(d)
            dist = rng.uniform(0.0, ra + rb + 0.2)
            vb = vb0 + _snap(dist * d, step)[None, :]
        fb = tf[:, ::-1].copy() if cls == 1 else tf
        A_list.append((_f32(va), tf))
        B_list.append((_f32(vb), fb))
        classes.append(cls_names[cls])
    pairs = np.stack([np.arange(n_pairs), np.arange(n_pairs)], 1).astype(np.int32)
    return concat_meshes(A_list), concat_meshes(B_list), pairs, classes


def make_c5_pool(seed: int = 5, n_meshes: int = 50_000, side: float = 58.5):
    """Serving pool: n_meshes C1-recipe meshes (level-2 icospheres, r~U[0.8,1.2],
    radial jitter N(0, 0.02 r)) with centres U[0, side]^3, split by id parity
    into R (even) and S (odd)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tv, tf = icosphere(2)
    meshes = []
    for _ in range(n_meshes):
        r = rng.uniform(0.8, 1.2)
        c = rng.uniform(0.0, side, size=3)
        meshes.append((_f32(_jittered_sphere(rng, tv, c, r, 0.02)), tf))
    return concat_meshes(meshes[0::2]), concat_meshes(meshes[1::2])


def _count_in_box(box_r: np.ndarray, box_s: np.ndarray, q: np.ndarray) -> int:
    """Pairs (r, s) whose closed boxes and the closed query box q share a
    point: used only to redraw query boxes of the serving trace."""
    sr = np.nonzero(np.all(box_r[:, :3] <= q[3:], 1) & np.all(box_r[:, 3:] >= q[:3], 1))[0]
    ss = np.nonzero(np.all(box_s[:, :3] <= q[3:], 1) & np.all(box_s[:, 3:] >= q[:3], 1))[0]
    if sr.size == 0 or ss.size == 0:
        return 0
    a, b = box_r[sr], box_s[ss]
    lo = np.maximum(np.maximum(a[:, None, :3], b[None, :, :3]), q[None, None, :3])
    hi = np.minimum(np.minimum(a[:, None, 3:], b[None, :, 3:]), q[None, None, 3:])
    return int(np.all(lo <= hi, axis=2).sum())


def c5_queries(box_r: np.ndarray, box_s: np.ndarray, n: int, lam: float, seed: int = 5, k_lo: float = 1.0,
               k_hi: float = 5000.0, space: float = 58.5, min_pairs: int = 1, max_pairs: int = 5000):
    """Serving trace: n requests with Poisson arrivals at rate lam (seconds
    from the start); each has a target size k ~ LogUniform[k_lo, k_hi] and a
    cubic query box of side k^(1/3) at a uniform centre in [0, space]^3,
    redrawn until it selects between min_pairs and max_pairs candidate pairs.
    Returns [(t_arrival, box f32[6])]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for _ in range(n):
        t += rng.exponential(1.0 / lam)
        while True:
            k = float(np.exp(rng.uniform(np.log(k_lo), np.log(k_hi))))
            side = k ** (1.0 / 3.0)
            c = rng.uniform(0.0, space, size=3)
            q = np.concatenate([c - side / 2, c + side / 2]).astype(np.float32)
            cnt = _count_in_box(box_r, box_s, q)
            if min_pairs <= cnt <= max_pairs:
                break
        out.append((t, q))
    return out


# ---------------------------------------------------------------------------
# Mesh-complexity sweep (Section 4.4, Fig. 3c)
# ---------------------------------------------------------------------------

def uv_sphere(rings: int, segments: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit latitude-longitude sphere: two poles and rings - 1 circles of
    `segments` vertices, V = (rings - 1) segments + 2, F = 2V - 4, faces
    outward (fans at the poles, split quads between circles)."""
    th = np.pi * np.arange(1, rings) / rings
    ph = 2 * np.pi * np.arange(segments) / segments
    ring = np.stack([np.sin(th)[:, None] * np.cos(ph)[None, :], np.sin(th)[:, None] * np.sin(ph)[None, :],
                     np.broadcast_to(np.cos(th)[:, None], (rings - 1, segments))], -1).reshape(-1, 3)
    v = np.concatenate([[[0.0, 0.0, 1.0]], ring, [[0.0, 0.0, -1.0]]])
    south = v.shape[0] - 1
    idx = lambda r, k: 1 + r * segments + (k % segments)  # noqa: E731
    f = []
    for k in range(segments):
        f.append([0, idx(0, k), idx(0, k + 1)])
        f.append([south, idx(rings - 2, k + 1), idx(rings - 2, k)])
        for r in range(rings - 2):
            a, b, c, d = idx(r, k), idx(r + 1, k), idx(r + 1, k + 1), idx(r, k + 1)
            f += [[a, b, c], [a, c, d]]
    return v, np.asarray(f, np.int32)


# rings of the five tessellation stages: (rings - 1) * 2 rings + 2 vertices =
# 26, 762, 2,966, 10,806, 41,186 (48 ... 82,368 triangles per sphere)
SWEEP_RINGS = (4, 20, 39, 74, 144)


def make_sweep(stage: int, seed: int = 6, n: int = 500, n_true: int = 100, side: float = 48.0):
    """Two datasets of n unit spheres at placements fixed across the
    tessellation stages (only the template changes).  n_true B spheres sit at
    distance U[0.3, 1.0] from a distinct A sphere (the surfaces cross at every
    stage: a translate of a convex body by 0 < d <= 1 is neither inside it nor
    apart from it, the coarsest template's inradius being above 1/2); every
    other centre distance between A and B is above 2.05 (apart at every stage:
    the vertices lie on the unit sphere), and a quarter of the remaining B
    spheres are placed at distance U[2.05, 3.2] from some A sphere, so that
    their boxes still overlap.  Returns (A, B)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ca = np.zeros((0, 3))
    while ca.shape[0] < n:               # A: centres at least 2.5 apart
        c = rng.uniform(0.0, side, size=3)
        if ca.shape[0] == 0 or np.min(np.linalg.norm(ca - c, axis=1)) > 2.5:
            ca = np.vstack([ca, c])
    cb = []

    def ok(c, partner):
        d = np.linalg.norm(ca - c, axis=1)
        if partner >= 0:
            d = np.delete(d, partner)
        far = d.min() > 2.05 if d.size else True
        return far and all(np.linalg.norm(c - x) > 2.05 for x in cb)

    partners = rng.choice(n, n_true, replace=False)
    for k in range(n):
        while True:
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            if k < n_true:
                p = int(partners[k])
                c = ca[p] + u * rng.uniform(0.3, 1.0)
            elif k < n_true + (n - n_true) // 4:
                p = -1
                c = ca[rng.integers(n)] + u * rng.uniform(2.05, 3.2)
            else:
                p = -1
                c = rng.uniform(0.0, side, size=3)
            if ok(c, p):
                cb.append(c)
                break
    tv, tf = uv_sphere(SWEEP_RINGS[stage], 2 * SWEEP_RINGS[stage])
    A = concat_meshes([(_f32(c[None, :] + tv), tf) for c in ca])
    B = concat_meshes([(_f32(c[None, :] + tv), tf) for c in np.asarray(cb)])
    return A, B


# ---------------------------------------------------------------------------
# Materialisation study (Section 4.6, Fig. 5): axis-aligned cubes
# ---------------------------------------------------------------------------

_CUBE_V = np.array([[x, y, z] for x in (0.0, 1.0) for y in (0.0, 1.0) for z in (0.0, 1.0)])
_CUBE_F = np.array([[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
                    [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]], np.int32)


def make_cubes(n: int = 50_000, side: float = 30.0, s_lo: float = 1.0, s_hi: float = 2.0, seed: int = 7):
    """Two datasets of n axis-aligned cubes (12 triangles each), sides
    U[s_lo, s_hi], lower corners uniform in [0, side]^3; the join selectivity
    is set by `side` (about ((2 mean side) / side)^3).  Returns (A, B)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(2):
        s = rng.uniform(s_lo, s_hi, size=n)
        c = rng.uniform(0.0, side, size=(n, 3))
        v = (c[:, None, :] + s[:, None, None] * _CUBE_V[None]).reshape(-1, 3)
        verts = _f32(v)
        faces = np.tile(_CUBE_F, (n, 1))
        vo = np.arange(n + 1, dtype=np.int64) * 8
        fo = np.arange(n + 1, dtype=np.int64) * 12
        out.append(MeshSet(verts, faces, vo, fo))
    return out[0], out[1]

