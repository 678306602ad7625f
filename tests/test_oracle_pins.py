"""Pins for the exact CPU oracle (no GPU).

The oracle decides closed triangle-triangle and mesh-pair intersection
(Section 3.2's overlap predicate read with closed sets).  It is pinned here
against things other than itself:
  * orientation signs against exact rational arithmetic (Fractions) and
    against plain FP64 on grids where FP64 is provably exact;
  * a second, independently written formulation of triangle-triangle
    intersection (edge-face form on exact rationals, tests/exact_ref.py);
  * scipy's LP solver on robustly decided random cases;
  * hand-built meshes whose answer follows from their construction
    (tests/golden/hand_cases.json);
  * closed-form mesh-level facts (ball separation, inside/outside vertices,
    nesting);
  * invariances of the definition (swap, permutation, winding, exact scaling,
    mirroring, exact translation);
  * planted mistakes in copies of the oracle source, each of which must be
    caught by these pins (test_planted_mistakes_are_caught).
"""
import ctypes
import json
import os
import subprocess
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import exact_ref  # noqa: E402

from paper_2609_24513_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _f32(x):
    return np.asarray(x, np.float32)


# ---------------------------------------------------------------------------
# orientation predicate
# ---------------------------------------------------------------------------

def _rand_wide_floats(rng, n):
    """FP32 values with widely spread exponents, signs, zeros and subnormals."""
    mant = rng.uniform(1.0, 2.0, size=n)
    ex = rng.integers(-140, 100, size=n)
    v = mant * np.power(2.0, ex.astype(np.float64))
    v *= np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    v[rng.uniform(size=n) < 0.05] = 0.0
    sub = rng.uniform(size=n) < 0.03
    v[sub] = rng.integers(1, 1 << 20, size=sub.sum()) * 2.0 ** -149
    return v.astype(np.float32)


def test_orient3d_matches_fractions_wide_exponents(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(400):
        pts = _rand_wide_floats(rng, 12).reshape(4, 3)
        ex = np.sign(float(exact_ref.orient3d(*[exact_ref.pt(p) for p in pts])))
        assert oracle_mod.orient3d(*pts) == ex


def test_orient3d_matches_fractions_near_degenerate(oracle_mod):
    rng = np.random.default_rng(12)
    for _ in range(400):
        a, b, c = rng.uniform(-3, 3, size=(3, 3))
        s, t = rng.uniform(-1, 2, size=2)
        d = a + s * (b - a) + t * (c - a)  # on the plane, then rounded to FP32
        pts = _f32([a, b, c, d])
        ex = exact_ref.orient3d(*[exact_ref.pt(p) for p in pts])
        assert oracle_mod.orient3d(*pts) == (ex > 0) - (ex < 0)


def test_orient3d_grid_exact_in_fp64(oracle_mod):
    """On a 2^-12 grid with |x| <= 4, every term of the 3x3 determinant is an
    integer multiple of 2^-36 below 2^48, so plain FP64 is exact there."""
    rng = np.random.default_rng(13)
    k = rng.integers(-5300, 5301, size=(3000, 4, 3))
    # many exact zeros: coplanar (d = b + c - a) and coincident points
    k[::3, 3] = k[::3, 1] + k[::3, 2] - k[::3, 0]
    k[1::7, 3] = k[1::7, 1]
    assert np.abs(k).max() <= 4 * 4096
    P = k.astype(np.float64) / 4096.0
    u = P[:, 1] - P[:, 0]; v = P[:, 2] - P[:, 0]; w = P[:, 3] - P[:, 0]
    det = (u[:, 0] * (v[:, 1] * w[:, 2] - v[:, 2] * w[:, 1])
           + u[:, 1] * (v[:, 2] * w[:, 0] - v[:, 0] * w[:, 2])
           + u[:, 2] * (v[:, 0] * w[:, 1] - v[:, 1] * w[:, 0]))
    zeros = 0
    for i in range(P.shape[0]):
        s = oracle_mod.orient3d(*_f32(P[i]))
        assert s == int(np.sign(det[i]))
        zeros += s == 0
    assert zeros > 300


def test_orient3d_identities(oracle_mod):
    rng = np.random.default_rng(14)
    for _ in range(200):
        a, b, c, d = _f32(rng.normal(size=(4, 3)))
        s = oracle_mod.orient3d(a, b, c, d)
        assert oracle_mod.orient3d(b, a, c, d) == -s      # odd permutation
        assert oracle_mod.orient3d(b, c, a, d) == s       # even permutation
        assert oracle_mod.orient3d(a, b, c, a) == 0       # repeated point
        assert oracle_mod.orient3d(a, a, c, d) == 0
    z = _f32(rng.normal(size=(4, 3)) * [1, 1, 0])        # all in z=0
    assert oracle_mod.orient3d(*z) == 0
    e = np.eye(3, dtype=np.float32)
    assert oracle_mod.orient3d(np.zeros(3, np.float32), e[0], e[1], e[2]) == 1


# ---------------------------------------------------------------------------
# triangle-triangle
# ---------------------------------------------------------------------------

def _nondegenerate(t):
    t = [exact_ref.pt(p) for p in t]
    n = exact_ref._cross(exact_ref._sub(t[1], t[0]), exact_ref._sub(t[2], t[0]))
    return any(x != 0 for x in n)


def _compare_tritri(oracle_mod, tris):
    n_true = 0
    for t, u in tris:
        if not (_nondegenerate(t) and _nondegenerate(u)):
            continue
        got = oracle_mod.tri_tri(t, u)
        ref = exact_ref.tri_tri_edges(t, u)
        assert got == ref, (t.tolist(), u.tolist())
        n_true += ref
    return n_true


def test_tritri_matches_edge_form_small_int_grid(oracle_mod):
    """Vertices in {0,1,2}^3: dense in touching, collinear and coplanar cases."""
    rng = np.random.default_rng(21)
    tris = [(_f32(rng.integers(0, 3, size=(3, 3))), _f32(rng.integers(0, 3, size=(3, 3))))
            for _ in range(2500)]
    n_true = _compare_tritri(oracle_mod, tris)
    assert 300 < n_true < 2400


def test_tritri_matches_edge_form_dyadic_grid(oracle_mod):
    rng = np.random.default_rng(22)
    tris = []
    for _ in range(1500):
        t = rng.integers(-8, 9, size=(3, 3)) / 8.0
        u = rng.integers(-8, 9, size=(3, 3)) / 8.0
        if rng.uniform() < 0.3:           # share a vertex or an edge point
            u[0] = t[rng.integers(0, 3)]
        if rng.uniform() < 0.2:           # coplanar: flatten both into z = t0.z
            t[:, 2] = t[0, 2]; u[:, 2] = t[0, 2]
        tris.append((_f32(t), _f32(u)))
    n_true = _compare_tritri(oracle_mod, tris)
    assert n_true > 200


def test_tritri_matches_edge_form_float(oracle_mod):
    rng = np.random.default_rng(23)
    tris = []
    for _ in range(600):
        t = rng.uniform(-1, 1, size=(3, 3))
        u = rng.uniform(-1, 1, size=(3, 3))
        if rng.uniform() < 0.3:   # u's first vertex rounded onto t's plane
            s, r = rng.uniform(0, 0.5, size=2)
            u[0] = t[0] + s * (t[1] - t[0]) + r * (t[2] - t[0])
        tris.append((_f32(t), _f32(u * rng.choice([1e-20, 1.0, 1e20]))
                     if rng.uniform() < 0.05 else _f32(u)))
    _compare_tritri(oracle_mod, tris)


def test_tritri_matches_linprog_on_robust_cases(oracle_mod):
    """Closed triangles meet iff the LP {sum l_i t_i = sum m_j u_j, l, m in the
    simplex} is feasible.  scipy decides robust cases: L-inf distance > 1e-6
    means disjoint; the triangles shrunk by 1% about their centroids meeting
    means the originals meet."""
    from scipy.optimize import linprog

    def dist(t, u):
        # vars: l0..2, m0..2, s ; minimise s
        c = np.zeros(7); c[6] = 1
        Aeq = np.zeros((2, 7)); Aeq[0, :3] = 1; Aeq[1, 3:6] = 1
        beq = np.ones(2)
        Aub, bub = [], []
        for k in range(3):
            row = np.zeros(7); row[:3] = t[:, k]; row[3:6] = -u[:, k]
            r1 = row.copy(); r1[6] = -1; Aub.append(r1); bub.append(0)
            r2 = -row; r2[6] = -1; Aub.append(r2); bub.append(0)
        res = linprog(c, A_ub=np.array(Aub), b_ub=bub, A_eq=Aeq, b_eq=beq,
                      bounds=[(0, None)] * 7, method="highs")
        assert res.status == 0
        return res.fun

    rng = np.random.default_rng(24)
    decided = {True: 0, False: 0}
    for _ in range(500):
        t = _f32(rng.uniform(0, 1, size=(3, 3)))
        u = _f32(rng.uniform(0, 1, size=(3, 3)))
        T, U = t.astype(np.float64), u.astype(np.float64)
        if dist(T, U) > 1e-6:
            exp = False
        else:
            sh = lambda x: x.mean(0) + 0.99 * (x - x.mean(0))  # noqa: E731
            if dist(sh(T), sh(U)) < 1e-10:
                exp = True
            else:
                continue
        assert oracle_mod.tri_tri(t, u) == exp
        decided[exp] += 1
    assert decided[True] > 50 and decided[False] > 50


def test_tritri_rejects_degenerate(oracle_mod):
    t = _f32([[0, 0, 0], [1, 1, 1], [2, 2, 2]])
    u = _f32([[0, 0, 0], [1, 0, 0], [0, 1, 0]])
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.tri_tri(t, u)


def test_tritri_degenerate_refused_before_any_early_out(oracle_mod):
    """A degenerate triangle is refused wherever it lies, including far from
    the other triangle (boxes separated on a coordinate axis)."""
    u = _f32([[0, 0, 0], [1, 0, 0], [0, 1, 0]])
    for t in (_f32([[50, 50, 50], [51, 51, 51], [53, 53, 53]]),     # collinear, far away
              _f32([[-9, 4, 2], [-9, 4, 2], [-7, 1, 0]]),            # repeated vertex
              _f32([[3, 3, 3], [3, 3, 3], [3, 3, 3]])):              # a point
        for a, b in ((t, u), (u, t)):
            with pytest.raises(oracle_mod.OracleError) as ei:
                oracle_mod.tri_tri(a, b)
            assert ei.value.code == oracle_mod.ORACLE_E_DEGENERATE


def _one_mesh(v, f):
    return synth.concat_meshes([(np.asarray(v, np.float64), np.asarray(f))])


def test_join_refuses_bad_meshes(oracle_mod):
    """Face ids must lie in [0, V) of their mesh and coordinates must be
    finite (argument errors); a mesh holding a degenerate triangle is refused
    for every pair, even when that triangle is far from the other mesh."""
    tet_v = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
    tet_f = [[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]]
    good = _one_mesh(tet_v, tet_f)
    near = _one_mesh(np.asarray(tet_v) + 0.25, tet_f)
    pairs = np.zeros((1, 2), np.int32)
    assert oracle_mod.join(good, near, pairs)[0] == 1
    last_ok = _one_mesh(tet_v, [[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2], [1, 2, 3]])
    assert oracle_mod.join(last_ok, near, pairs)[0] == 1          # id V-1 is fine
    bad = {
        "id_equal_to_V": _one_mesh(tet_v, tet_f + [[1, 2, 4]]),
        "negative_id": _one_mesh(tet_v, tet_f + [[1, -1, 2]]),
        "nan": _one_mesh(tet_v[:3] + [[0, np.nan, 1]], tet_f),
        "inf": _one_mesh(tet_v[:3] + [[np.inf, 0, 1]], tet_f),
    }
    for name, m in bad.items():
        for a, b in ((m, near), (near, m)):
            with pytest.raises(oracle_mod.OracleError) as ei:
                oracle_mod.join(a, b, pairs)
            assert ei.value.code == -1, name
    far_deg = _one_mesh(tet_v + [[90, 90, 90], [91, 91, 91], [93, 93, 93]], tet_f + [[4, 5, 6]])
    for mode in (0, 1):
        for a, b in ((far_deg, near), (near, far_deg)):
            with pytest.raises(oracle_mod.OracleError) as ei:
                oracle_mod.join(a, b, pairs, mode=mode)
            assert ei.value.code == oracle_mod.ORACLE_E_DEGENERATE


def _extreme_pairs(rng, n):
    """Triangle pairs whose coordinates span the whole FP32 range, from the
    smallest subnormal to the largest finite value, with touching cases."""
    big = np.float32(np.finfo(np.float32).max)
    tiny = np.float32(2.0 ** -149)
    out = []
    for k in range(n):
        t = rng.uniform(-1, 1, size=(3, 3))
        u = rng.uniform(-1, 1, size=(3, 3))
        t[0] *= 2.0 ** 127 * rng.uniform(0.5, 1.0)
        u[1] = t[1]                                    # shared vertex: touching
        u[2] = [tiny, -tiny, 0.0] if k % 2 else [big, -big, tiny]
        out.append((_f32(t), _f32(u)))
    return out


def test_full_width_integers_cover_fp32_range(oracle_mod):
    """1280-bit integers hold every degree-4 product over the FP32 exponent
    range: extreme inputs decide without overflow and agree with exact
    rationals."""
    rng = np.random.default_rng(25)
    n = 0
    for t, u in _extreme_pairs(rng, 24):
        if not (_nondegenerate(t) and _nondegenerate(u)):
            continue
        assert oracle_mod.tri_tri(t, u) == exact_ref.tri_tri_edges(t, u)
        n += 1
    assert n >= 16


def test_overflow_is_reported_not_guessed(oracle_mod):
    """With the integer width lowered on purpose, values that do not fit are
    reported as an overflow error (single tests and mesh joins), never
    answered; the full width then answers the same inputs."""
    t = _f32([[0, 0, 0], [3, 0, 0], [0, 3, 0]])
    u = _f32([[1, 1, -1], [1, 1, 1], [2, 0.5, 1]])
    A, B = synth.make_c1(n=2)
    pairs = np.array([[0, 0], [1, 1]], np.int32)
    prev = oracle_mod.set_limb_budget(2)
    try:
        with pytest.raises(oracle_mod.OracleError) as ei:
            oracle_mod.tri_tri(t, u)
        assert ei.value.code == oracle_mod.ORACLE_E_OVERFLOW
        # exponents 80 bits apart: every scaled coordinate needs two limbs
        w = _f32([[0, 0, 0], [2.0 ** 40, 0, 0], [0, 2.0 ** 40, 0], [2.0 ** -40, 2.0 ** -40, 2.0 ** -40]])
        with pytest.raises(oracle_mod.OracleError) as ei:
            oracle_mod.orient3d(*w)
        assert ei.value.code == oracle_mod.ORACLE_E_OVERFLOW
        with pytest.raises(oracle_mod.OracleError) as ei:
            oracle_mod.join(A, B, np.array([[0, 0]], np.int32), mode=0)
        assert ei.value.code == oracle_mod.ORACLE_E_OVERFLOW
    finally:
        oracle_mod.set_limb_budget(prev)
    assert prev == 20
    assert oracle_mod.tri_tri(t, u) is True
    assert oracle_mod.orient3d(*w) == 1
    oracle_mod.join(A, B, pairs)


# ---------------------------------------------------------------------------
# candidate filter and unique edges (oracle/filter.py)
# ---------------------------------------------------------------------------

def _boxes_brute(S):
    out = []
    for m in range(S.n_meshes):
        v, f = S.mesh(m)
        if f.shape[0] == 0:
            out.append([np.inf] * 3 + [-np.inf] * 3)
            continue
        lo = [min(float(v[i][k]) for tri in f for i in tri) for k in range(3)]
        hi = [max(float(v[i][k]) for tri in f for i in tri) for k in range(3)]
        out.append(lo + hi)
    return np.array(out, np.float32)


def _pairs_brute(ba, bb, q=None):
    out = []
    for i in range(ba.shape[0]):
        for j in range(bb.shape[0]):
            ok = True
            for k in range(3):
                lo = max(ba[i][k], bb[j][k]) if q is None else max(ba[i][k], bb[j][k], q[k])
                hi = min(ba[i][3 + k], bb[j][3 + k]) if q is None else min(ba[i][3 + k], bb[j][3 + k], q[3 + k])
                ok = ok and lo <= hi
            if ok:
                out.append((i, j))
    return np.array(out, np.int64).reshape(-1, 2)


def test_filter_definition_brute_force(oracle_mod):
    """Closed-box candidates against a pure-Python double loop, on boxes that
    touch exactly (shared faces, edges, corners), miss by one ulp, nest, and
    with query boxes; mesh boxes against a loop over face vertices (unused
    vertices do not count, empty meshes have no box)."""
    rng = np.random.default_rng(41)
    for trial in range(6):
        na, nb = rng.integers(1, 25, size=2)
        lo = rng.integers(0, 6, size=(na + nb, 3)).astype(np.float32)
        hi = lo + rng.integers(0, 3, size=(na + nb, 3)).astype(np.float32)
        bx = np.concatenate([lo, hi], 1)
        # one-ulp misses and exact touches
        nudge = rng.uniform(size=na + nb) < 0.2
        bx[nudge, 3] = np.nextafter(bx[nudge, 3], np.float32(-np.inf))
        ba, bb = bx[:na], bx[na:]
        assert np.array_equal(oracle_mod.candidate_pairs(ba, bb), _pairs_brute(ba, bb))
        q = np.array([1, 0.5, 2, 3, 4, 3.5], np.float32)
        assert np.array_equal(oracle_mod.candidate_pairs(ba, bb, q), _pairs_brute(ba, bb, q))
    tet_f = [[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]]
    meshes = [(rng.uniform(-2, 2, size=(5, 3)), tet_f) for _ in range(6)]   # vertex 4 unused
    meshes.append((np.zeros((0, 3)), np.zeros((0, 3), np.int64)))          # empty mesh
    S = synth.concat_meshes(meshes)
    got = oracle_mod.mesh_boxes(S)
    assert np.array_equal(got, _boxes_brute(S))
    assert np.all(np.isinf(got[-1]))
    # an empty mesh is never a candidate, even against an infinite query box
    cand = oracle_mod.candidate_pairs(got, got, np.array([-np.inf] * 3 + [np.inf] * 3, np.float32))
    assert not np.any(cand == S.n_meshes - 1)
    assert cand.shape[0] >= 6


def test_unique_edges_closed_forms(oracle_mod):
    """Closed genus-0 triangle meshes: every edge is shared by two faces, so
    E = 3F/2, and Euler's formula V - E + F = 2 holds; icosphere level k has
    E = 30 * 4^k."""
    cases = [synth.icosphere(k) for k in (0, 1, 2, 4)]
    cases += [synth.geodesic_sphere(nu) for nu in (2, 5, 9)]
    ctrl = np.array([[0, 0, 0], [1, 2, 0], [3, 1, 1], [4, 4, 2]], np.float64)
    cases += [synth.capped_tube(ctrl, 0.5, r, s) for r, s in ((2, 4), (64, 32), (7, 11))]
    for k, (v, f) in enumerate(cases):
        e = oracle_mod.unique_edges(f)
        F, V = f.shape[0], v.shape[0]
        assert 2 * e.shape[0] == 3 * F, k
        assert V - e.shape[0] + F == 2, k
        assert np.all(e[:, 0] < e[:, 1])
    for lvl in (0, 1, 2, 4):
        assert oracle_mod.unique_edges(synth.icosphere(lvl)[1]).shape[0] == 30 * 4 ** lvl
    # a lone triangle has three edges; the same edge in both orientations counts once
    assert oracle_mod.unique_edges(np.array([[0, 1, 2]])).tolist() == [[0, 1], [0, 2], [1, 2]]
    assert oracle_mod.unique_edges(np.array([[0, 1, 2], [2, 1, 3]])).shape[0] == 5


# ---------------------------------------------------------------------------
# mesh level
# ---------------------------------------------------------------------------

def _hand_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as fh:
        return json.load(fh)["cases"]


def _single(m):
    return synth.concat_meshes([(np.asarray(m["verts"], np.float64), np.asarray(m["faces"]))])


@pytest.mark.parametrize("mode", [0, 1])
def test_hand_built_cases(oracle_mod, mode):
    cases = _hand_cases()
    A = synth.concat_meshes([(np.asarray(c["A"]["verts"], np.float64), np.asarray(c["A"]["faces"])) for c in cases])
    B = synth.concat_meshes([(np.asarray(c["B"]["verts"], np.float64), np.asarray(c["B"]["faces"])) for c in cases])
    pairs = np.stack([np.arange(len(cases))] * 2, 1)
    got = oracle_mod.join(A, B, pairs, mode=mode)
    exp = np.array([c["expected"] for c in cases], np.uint8)
    bad = [cases[i]["name"] for i in np.nonzero(got != exp)[0]]
    assert not bad, bad
    # swapped roles give the same answers
    got2 = oracle_mod.join(B, A, pairs, mode=mode)
    assert np.array_equal(got2, exp)


def _pin_pairs(seed=31, n=300):
    """Level-2 jittered icospheres (the tiny config's recipe), with B's centre
    at a random distance from A's so that many pairs straddle A's surface."""
    rng = np.random.default_rng(seed)
    tv, tf = synth.icosphere(2)
    As, Bs, info = [], [], []
    for _ in range(n):
        ra, rb = rng.uniform(0.8, 1.2, size=2)
        ca = rng.uniform(0, 4, size=3)
        d = rng.normal(size=3); d /= np.linalg.norm(d)
        cb = ca + d * rng.uniform(0.0, 2.8)
        va = (ca[None] + (ra + rng.normal(0, 0.02 * ra, size=162))[:, None] * tv).astype(np.float32)
        vb = (cb[None] + (rb + rng.normal(0, 0.02 * rb, size=162))[:, None] * tv).astype(np.float32)
        As.append((va, tf)); Bs.append((vb, tf)); info.append((ca, cb))
    return synth.concat_meshes(As), synth.concat_meshes(Bs), info


def _radii(v, f, c):
    """(rho, R): rho is a lower bound of the distance from c to the surface
    (distance to the nearest face plane), R the largest vertex distance."""
    v = v.astype(np.float64)
    a, b, cc = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(b - a, cc - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    rho = np.abs(np.einsum("ij,ij->i", n, a - c[None])).min()
    R = np.linalg.norm(v - c[None], axis=1).max()
    return rho, R


def test_mesh_level_closed_forms(oracle_mod):
    """A and B are star-shaped about their generating centres c (radial
    graphs), so c is inside; the open ball of radius rho about c lies inside
    the solid, and everything beyond R lies outside.
      |cA-cB| > RA+RB                            => FALSE (disjoint balls)
      all of B within rho_A of cA (or A of B)    => FALSE (strictly nested)
      B has a vertex within rho_A and one beyond R_A (or vice versa)
                                                 => TRUE (a connected surface
                                                    going from inside to outside)"""
    A, B, info = _pin_pairs()
    pairs = np.stack([np.arange(A.n_meshes)] * 2, 1)
    got = oracle_mod.join(A, B, pairs, mode=1)
    m = 1e-9
    labelled = {True: 0, False: 0}
    for i, (ca, cb) in enumerate(info):
        va, fa = A.mesh(i); vb, fb = B.mesh(i)
        rA, RA = _radii(va, fa, ca)
        rB, RB = _radii(vb, fb, cb)
        dB = np.linalg.norm(vb.astype(np.float64) - ca[None], axis=1)
        dA = np.linalg.norm(va.astype(np.float64) - cb[None], axis=1)
        lab = None
        if np.linalg.norm(ca - cb) > (RA + RB) * (1 + m):
            lab = False
        elif dB.max() < rA * (1 - m) or dA.max() < rB * (1 - m):
            lab = False
        elif (dB.min() < rA * (1 - m) and dB.max() > RA * (1 + m)) or \
             (dA.min() < rB * (1 - m) and dA.max() > RB * (1 + m)):
            lab = True
        if lab is not None:
            assert bool(got[i]) == lab, i
            labelled[lab] += 1
    assert labelled[True] >= 40 and labelled[False] >= 40, labelled


def test_brute_force_equals_pruned_c1(oracle_mod):
    A, B = synth.make_c1()
    pairs = np.array([(i, j) for i in range(8) for j in range(8)], np.int32)
    f0 = oracle_mod.join(A, B, pairs, mode=0)
    f1 = oracle_mod.join(A, B, pairs, mode=1)
    assert np.array_equal(f0, f1)
    assert 5 < f0.sum() < 60


def test_brute_force_equals_pruned_c4_sample(oracle_mod):
    A, B, pairs, cls = synth.make_c4(n_pairs=40)
    f0 = oracle_mod.join(A, B, pairs, mode=0)
    f1 = oracle_mod.join(A, B, pairs, mode=1)
    assert np.array_equal(f0, f1)
    # contact constructions come out TRUE under closed semantics
    for k, c in enumerate(cls):
        if c in ("tangent", "coplanar", "on_surface"):
            assert f1[k] == 1, (k, c)


def _transform(S, fn_v=None, fn_f=None):
    v = S.verts if fn_v is None else fn_v(S.verts)
    f = S.faces if fn_f is None else fn_f(S.faces)
    return synth.MeshSet(np.ascontiguousarray(v.astype(np.float32)), np.ascontiguousarray(f.astype(np.int32)),
                         S.vert_off.copy(), S.face_off.copy())


def test_metamorphic_invariances(oracle_mod):
    A, B = synth.make_c1(seed=7)
    pairs = np.array([(i, j) for i in range(8) for j in range(8)], np.int32)
    base = oracle_mod.join(A, B, pairs)
    # swap roles
    sw = oracle_mod.join(B, A, pairs[:, ::-1].copy())
    assert np.array_equal(sw, base)
    # exact transforms applied to both datasets
    for fv in (lambda v: v * np.float32(2.0 ** 7), lambda v: v * np.float32(2.0 ** -9),
               lambda v: v * np.array([-1, 1, 1], np.float32), lambda v: v[:, [2, 0, 1]]):
        assert np.array_equal(oracle_mod.join(_transform(A, fv), _transform(B, fv), pairs), base)
    # winding and triangle order
    rev = lambda f: f[:, ::-1]  # noqa: E731
    assert np.array_equal(oracle_mod.join(_transform(A, fn_f=rev), B, pairs), base)
    rng = np.random.default_rng(3)
    fperm = []
    for m in range(A.n_meshes):
        lo, hi = A.face_off[m], A.face_off[m + 1]
        fperm.append(lo + rng.permutation(hi - lo))
    fperm = np.concatenate(fperm)
    assert np.array_equal(oracle_mod.join(_transform(A, fn_f=lambda f: f[fperm]), B, pairs), base)


def test_metamorphic_exact_translation_on_grid(oracle_mod):
    A, B, pairs, _ = synth.make_c4(n_pairs=30)
    base = oracle_mod.join(A, B, pairs)
    t = np.array([1.0, -0.5, 0.25], np.float32)
    At, Bt = _transform(A, lambda v: v + t), _transform(B, lambda v: v + t)
    assert np.all((At.verts - t) == A.verts)  # translation was exact
    assert np.array_equal(oracle_mod.join(At, Bt, pairs), base)


# ---------------------------------------------------------------------------
# planted mistakes: each must be caught by the pins above
# ---------------------------------------------------------------------------

MUTANTS = {
    "open_semantics": ("if (cmp(mx(pt), mn(pu)) < 0) return true;", "if (cmp(mx(pt), mn(pu)) <= 0) return true;"),
    "no_edge_cross_axes": ("if (!is_zero(L) && separates(L, T, U)) return 0;", "(void)L;"),
    "no_inplane_axes": ("    V3 L = cross(nt, et[i]);\n    if (separates(L, T, U)) return 0;\n    L = cross(nu, eu[i]);\n    if (separates(L, T, U)) return 0;",
                        "    (void)i;"),
    "cross_sign": ("return {sub(mul(a.y, b.z), mul(a.z, b.y)),", "return {sub(mul(a.z, b.y), mul(a.y, b.z)),"),
    "lost_low_bits": ("std::ldexp((double)std::fabs(f), 24)", "std::floor(std::ldexp((double)std::fabs(f), 20))"),
    "borrow_dropped": ("uint64_t t = a.d[i] - bi - borrow;", "uint64_t t = a.d[i] - bi;"),
    "face_id_off_by_one": ("if (m.f[i] < 0 || m.f[i] >= m.nv) return false;",
                           "if (m.f[i] < 0 || m.f[i] > m.nv) return false;"),
    "nonfinite_accepted": ("if (!std::isfinite(m.v[i])) return false;", "if (std::isnan(m.v[i])) return false;"),
    "degenerate_checked_late": ("  if (tri_degenerate(t) || tri_degenerate(u)) return ORACLE_E_DEGENERATE;\n  return tri_tri_core(t, u);",
                                "  int r = tri_tri_core(t, u);\n  if (r && (tri_degenerate(t) || tri_degenerate(u))) return ORACLE_E_DEGENERATE;\n  return r;"),
    "mesh_degeneracy_skipped": ("v = mesh_degenerate(m) == 0 ? 1 : 2;", "v = 1;"),
    "too_few_limbs": ("constexpr int LIMBS = 20;", "constexpr int LIMBS = 12;"),
    "overflow_not_reported": ("if (a.n + b.n > limb_budget()) { g_overflow = true; return r; }",
                              "if (a.n + b.n > LIMBS) { g_overflow = true; return r; }"),
}


def _load_variant(path):
    lib = ctypes.CDLL(path)
    fp = ctypes.POINTER(ctypes.c_float)
    ip = ctypes.POINTER(ctypes.c_int32)
    lp = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_tri_tri.argtypes = [fp, fp]
    lib.oracle_orient3d.argtypes = [fp, fp, fp, fp]
    lib.oracle_join.argtypes = [fp, ip, lp, lp, ctypes.c_int64, fp, ip, lp, lp, ctypes.c_int64,
                                ip, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_set_limb_budget.argtypes = [ctypes.c_int]
    return lib


def _variant_join(lib, A, B, pairs, mode=1):
    """oracle_join of a compiled variant: (return code, flags)."""
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    flags = np.zeros(pairs.shape[0], np.uint8)
    args = []
    keep = []
    for S in (A, B):
        v = np.ascontiguousarray(S.verts, np.float32); f = np.ascontiguousarray(S.faces, np.int32)
        vo = np.ascontiguousarray(S.vert_off, np.int64); fo = np.ascontiguousarray(S.face_off, np.int64)
        keep += [v, f, vo, fo]
        args += [v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                 vo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), fo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                 ctypes.c_int64(vo.shape[0] - 1)]
    n = ctypes.c_uint64(0)
    r = lib.oracle_join(*args, pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.c_int64(pairs.shape[0]),
                        flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.c_int(mode), ctypes.c_int(1),
                        ctypes.byref(n))
    return r, flags


def _variant_pins_pass(lib):
    """A quick subset of the pins, run against a compiled variant."""
    fp = ctypes.POINTER(ctypes.c_float)

    def tt(t, u):
        t = np.ascontiguousarray(_f32(t).reshape(9)); u = np.ascontiguousarray(_f32(u).reshape(9))
        return lib.oracle_tri_tri(t.ctypes.data_as(fp), u.ctypes.data_as(fp))

    def o3(*p):
        p = [np.ascontiguousarray(_f32(x)) for x in p]
        return lib.oracle_orient3d(*[x.ctypes.data_as(fp) for x in p])

    rng = np.random.default_rng(5)
    for _ in range(150):
        pts = _rand_wide_floats(rng, 12).reshape(4, 3)
        ex = exact_ref.orient3d(*[exact_ref.pt(p) for p in pts])
        if o3(*pts) != (ex > 0) - (ex < 0):
            return False
    for _ in range(150):   # points rounded onto a plane
        a, b, c = rng.uniform(-3, 3, size=(3, 3))
        s, r = rng.uniform(-1, 2, size=2)
        pts = _f32([a, b, c, a + s * (b - a) + r * (c - a)])
        ex = exact_ref.orient3d(*[exact_ref.pt(p) for p in pts])
        if o3(*pts) != (ex > 0) - (ex < 0):
            return False
    for _ in range(400):
        t = _f32(rng.integers(0, 3, size=(3, 3))); u = _f32(rng.integers(0, 3, size=(3, 3)))
        if not (_nondegenerate(t) and _nondegenerate(u)):
            continue
        if bool(tt(t, u)) != exact_ref.tri_tri_edges(t, u):
            return False
    for _ in range(200):
        t = _f32(rng.uniform(-1, 1, size=(3, 3))); u = _f32(rng.uniform(-1, 1, size=(3, 3)))
        if bool(tt(t, u)) != exact_ref.tri_tri_edges(t, u):
            return False
    for _ in range(300):   # coplanar pairs on a dyadic grid
        t = rng.integers(-8, 9, size=(3, 3)) / 8.0; u = rng.integers(-8, 9, size=(3, 3)) / 8.0
        t[:, 2] = 0.0; u[:, 2] = 0.0
        t, u = _f32(t), _f32(u)
        if not (_nondegenerate(t) and _nondegenerate(u)):
            continue
        if bool(tt(t, u)) != exact_ref.tri_tri_edges(t, u):
            return False
    for t, u in _extreme_pairs(np.random.default_rng(25), 24):   # whole FP32 range
        if not (_nondegenerate(t) and _nondegenerate(u)):
            continue
        if tt(t, u) != int(exact_ref.tri_tri_edges(t, u)):
            return False
    # a degenerate triangle far away is refused, not answered
    if tt(_f32([[50, 50, 50], [51, 51, 51], [53, 53, 53]]), _f32([[0, 0, 0], [1, 0, 0], [0, 1, 0]])) != -3:
        return False
    # mesh-level argument checks and degenerate meshes
    tet_v = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
    tet_f = [[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]]
    near = _one_mesh(np.asarray(tet_v) + 0.25, tet_f)
    pr = np.zeros((1, 2), np.int32)
    r, f = _variant_join(lib, _one_mesh(tet_v, tet_f), near, pr)
    if r != 0 or f[0] != 1:
        return False
    for m in (_one_mesh(tet_v, tet_f + [[1, 2, 4]]), _one_mesh(tet_v[:3] + [[np.inf, 0, 1]], tet_f)):
        if _variant_join(lib, m, near, pr)[0] != -1:
            return False
    far_deg = _one_mesh(tet_v + [[90, 90, 90], [91, 91, 91], [93, 93, 93]], tet_f + [[4, 5, 6]])
    if _variant_join(lib, far_deg, near, pr)[0] != -3:
        return False
    # lowered integer width: overflow reported
    lib.oracle_set_limb_budget(2)
    r = tt(_f32([[0, 0, 0], [3, 0, 0], [0, 3, 0]]), _f32([[1, 1, -1], [1, 1, 1], [2, 0.5, 1]]))
    lib.oracle_set_limb_budget(20)
    if r != -6:
        return False
    return True


@pytest.mark.slow
def test_planted_mistakes_are_caught(tmp_path, oracle_mod):
    src = open(os.path.join(ROOT, "oracle", "oracle.cpp")).read()
    # the unmodified source passes the quick pins
    ok_so = str(tmp_path / "orig.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread", "-x", "c++", "-", "-o", ok_so],
                          input=src.encode(), check=True)
    assert _variant_pins_pass(_load_variant(ok_so))
    for name, (old, new) in MUTANTS.items():
        assert old in src, name
        so = str(tmp_path / (name + ".so"))
        subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread", "-x", "c++", "-", "-o", so],
                              input=src.replace(old, new).encode(), check=True)
        assert not _variant_pins_pass(_load_variant(so)), name
