"""Pins for the oracle's selectivity estimate (Section 3.5), with no GPU.

The estimate is a model, so it is pinned to what its parts mean rather than
to itself: mesh volumes against closed forms; the interaction-volume
probability against the overlap frequency of many uniformly placed cubes
(Monte Carlo, the Minkowski-sum argument); the shape factor against
octahedra, whose volume is a sixth of their box; the cap; and invariances
(swap, permutation, scaling).
"""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
from containment_inputs import CUBE_V, CUBE_F, OCT_V, OCT_F, TET_V, TET_F, mesh_set  # noqa: E402

from paper_2609_24513_amd import synth  # noqa: E402


def _est(oracle_mod, A, B, cells=8):
    return oracle_mod.estimate.estimate(A, B, oracle_mod.mesh_boxes(A), oracle_mod.mesh_boxes(B), cells)


def test_mesh_volumes_closed_forms(oracle_mod):
    S = mesh_set((CUBE_V, CUBE_F), (TET_V, TET_F), (OCT_V, OCT_F), (np.asarray(CUBE_V) * 2 + 1000, CUBE_F),
                 (CUBE_V, np.asarray(CUBE_F)[:, ::-1]))
    v = oracle_mod.estimate.mesh_volumes(S)
    assert np.allclose(v, [1.0, 1.0 / 6.0, 4.0 / 3.0, 8.0, 1.0], rtol=1e-9, atol=0)
    tv, tf = synth.icosphere(4)
    ico = oracle_mod.estimate.mesh_volumes(mesh_set((3.0 * tv, tf)))[0]
    ball = 4.0 / 3.0 * np.pi * 27.0
    assert 0.99 * ball < ico < ball      # inscribed polyhedron, 5,120 faces


def _cubes(rng, n, side, lo, hi):
    ms = []
    for _ in range(n):
        s = rng.uniform(*side)
        c = rng.uniform(lo, hi, size=3)
        ms.append((c + s * (np.asarray(CUBE_V, np.float64) - 0.5), CUBE_F))
    return synth.concat_meshes(ms)


def test_interaction_volume_matches_overlap_frequency(oracle_mod):
    """One cell; cubes of side s ~ U[0.8, 1.2] with centres uniform in
    [0, 40]^3: the estimate N1 N2 ((S1 + S2 + eps) / L)^3 against the number
    of box-overlapping pairs counted by brute force (boundary effects make
    the count a few percent lower, the spread of the sides a few percent
    higher)."""
    rng = np.random.default_rng(8)
    A = _cubes(rng, 3000, (0.8, 1.2), 0.0, 40.0)
    B = _cubes(rng, 3000, (0.8, 1.2), 0.0, 40.0)
    r = _est(oracle_mod, A, B, cells=1)
    # the cell is the union of the boxes, one side wider than the centres'
    # range [0, 40]: rescale to the centres' range before comparing
    e = r["estimate"] * float(np.prod(r["cell_size"])) / 40.0 ** 3
    ba, bb = oracle_mod.mesh_boxes(A).astype(np.float64), oracle_mod.mesh_boxes(B).astype(np.float64)
    count = 0
    for k in range(ba.shape[0]):
        ov = np.all((ba[k, :3] <= bb[:, 3:]) & (bb[:, :3] <= ba[k, 3:]), axis=1)
        count += int(ov.sum())
    assert count > 500
    assert 0.92 < count / e < 1.08, (count, e)


def test_shape_factor_from_volumes(oracle_mod):
    """Octahedra fill a sixth of their box: with the same boxes, the estimate
    for octahedra is (1/6)^0.8 times the estimate for cubes (all cells below
    the cap)."""
    rng = np.random.default_rng(9)
    cen_a = rng.uniform(0, 30, size=(400, 3))
    cen_b = rng.uniform(0, 30, size=(400, 3))

    def build(shape_v, shape_f, cen, half):
        return synth.concat_meshes([(c + half * np.asarray(shape_v, np.float64), shape_f) for c in cen])

    cube_c = np.asarray(CUBE_V, np.float64) * 2.0 - 1.0     # [-1, 1]^3, as the octahedron's box
    Ac, Bc = build(cube_c, CUBE_F, cen_a, 0.5), build(cube_c, CUBE_F, cen_b, 0.5)
    Ao, Bo = build(OCT_V, OCT_F, cen_a, 0.5), build(OCT_V, OCT_F, cen_b, 0.5)
    ec, eo = _est(oracle_mod, Ac, Bc)["estimate"], _est(oracle_mod, Ao, Bo)["estimate"]
    assert ec > 0
    assert eo / ec == pytest.approx((1.0 / 6.0) ** 0.8, rel=1e-9)


def test_cap_at_one(oracle_mod):
    """Objects larger than the cell: every cell's probability is 1, so a
    single cell holds N1 N2 expected pairs."""
    rng = np.random.default_rng(10)
    A = _cubes(rng, 7, (5.0, 5.0), 0.0, 1.0)
    B = _cubes(rng, 5, (5.0, 5.0), 0.0, 1.0)
    assert _est(oracle_mod, A, B, cells=1)["estimate"] == pytest.approx(35.0, rel=1e-12)


def test_invariances(oracle_mod):
    rng = np.random.default_rng(11)
    A = _cubes(rng, 300, (0.5, 2.0), 0.0, 20.0)
    B = _cubes(rng, 200, (0.5, 2.0), 0.0, 20.0)
    e = _est(oracle_mod, A, B)["estimate"]
    assert _est(oracle_mod, B, A)["estimate"] == pytest.approx(e, rel=1e-12)
    perm = rng.permutation(A.n_meshes)
    assert _est(oracle_mod, A.subset(perm), B)["estimate"] == pytest.approx(e, rel=1e-12)
    scale = lambda S: synth.MeshSet(S.verts * np.float32(4.0), S.faces, S.vert_off, S.face_off)  # noqa: E731
    # exact scaling by 4 leaves every ratio unchanged except the additive eps
    assert _est(oracle_mod, scale(A), scale(B))["estimate"] == pytest.approx(e, rel=5e-3)


def test_grid_counts_touching_boxes(oracle_mod):
    """A box on a cell boundary touches both cells (closed cells): two unit
    cubes in a 2-cell-wide grid, one straddling the middle plane."""
    A = mesh_set((np.asarray(CUBE_V, np.float64) * 2.0, CUBE_F))               # [0, 2]^3: the grid
    B = mesh_set((np.asarray(CUBE_V, np.float64) * 0.5 + [0.75, 0.0, 0.0], CUBE_F))  # x in [0.75, 1.25]
    r = _est(oracle_mod, A, B, cells=2)
    # B touches the 2 x 1 x 1 cells with y, z in [0, 1]; A touches all 8; per cell
    # P = min(((2 + 0.5 + eps) / 1)^3 ..., 1) = 1
    assert r["estimate"] == pytest.approx(2.0, rel=1e-12)
