"""The mesh-complexity sweep inputs (Section 4.4): template counts, and the
placement facts that make the result 100 pairs at every stage, checked on
the CPU (the oracle confirms them at the coarsest stage)."""
import numpy as np
import pytest

from paper_2609_24513_amd import synth

PAPER_VERTS = (26, 762, 2966, 10806, 41186)


@pytest.mark.parametrize("stage", range(5))
def test_uv_sphere_template(stage):
    m = synth.SWEEP_RINGS[stage]
    v, f = synth.uv_sphere(m, 2 * m)
    assert v.shape[0] == PAPER_VERTS[stage] and f.shape[0] == 2 * v.shape[0] - 4
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    # closed 2-manifold: every edge in exactly two faces, once in each direction
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    assert len({tuple(x) for x in e.tolist()}) == e.shape[0]
    assert {tuple(x) for x in e.tolist()} == {tuple(x) for x in e[:, ::-1].tolist()}
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    assert np.all(np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0)   # outward


def test_placement_facts():
    A, B = synth.make_sweep(0)
    ca = np.array([A.mesh(k)[0].astype(np.float64).mean(0) for k in range(A.n_meshes)])
    cb = np.array([B.mesh(k)[0].astype(np.float64).mean(0) for k in range(B.n_meshes)])
    d = np.linalg.norm(ca[:, None] - cb[None], axis=2)
    close = d < 2.05
    assert close.sum() == 100 and np.all(d[close] > 0.29) and np.all(d[close] < 1.01)
    assert np.all(close.sum(0) <= 1) and np.all(close.sum(1) <= 1)
    # every stage keeps the placements: the centres of the templates coincide
    A4, B4 = synth.make_sweep(4)
    cb4 = np.array([B4.mesh(k)[0].astype(np.float64).mean(0) for k in range(B4.n_meshes)])
    assert np.allclose(cb4, cb, atol=1e-5)


def test_coarsest_stage_oracle(oracle_mod):
    A, B = synth.make_sweep(0)
    pairs = oracle_mod.candidate_pairs(oracle_mod.mesh_boxes(A), oracle_mod.mesh_boxes(B))
    flags = oracle_mod.join(A, B, pairs)
    ca = np.array([A.mesh(k)[0].astype(np.float64).mean(0) for k in range(A.n_meshes)])
    cb = np.array([B.mesh(k)[0].astype(np.float64).mean(0) for k in range(B.n_meshes)])
    d = np.linalg.norm(ca[pairs[:, 0]] - cb[pairs[:, 1]], axis=1)
    assert flags.sum() == 100 and np.array_equal(flags.astype(bool), d < 2.05)
    assert pairs.shape[0] > 150     # near misses reach the refinement
