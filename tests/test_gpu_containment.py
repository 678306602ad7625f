"""GPU parity of the point-in-mesh test and the containment, within and
intersection predicates (inside_pairs / refine_predicate through the C ABI)
against the exact CPU oracle.

The raw bits (representative vertex inside / on the other surface, both
directions) have one correct value per pair and are compared bit for bit,
as are the four predicates.  Cases: hand-built nested and contact pairs,
lattice probes against a cube, a tetrahedron and an octahedron (rays along
edges, through vertices, in face planes), a torus, dyadic-grid nested
shapes, jittered spheres at every BVH width, a deep tree that overflows the
fast kernel's stack, sampled pairs of the pathology-shaped pool at full size,
argument errors and empty inputs.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import containment_inputs as ci  # noqa: E402


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import oracle
    oracle.build(force=False)
    import paper_2609_24513_amd as pa
    return torch, pa, oracle


def _blobs(pa, A, B, width=4, leaf=4):
    return pa.MeshBlob.build(A, width=width, leaf_size=leaf), pa.MeshBlob.build(B, width=width, leaf_size=leaf)


def _bits(env, ga, gb, pairs):
    torch, pa, oracle = env
    out, st, status = pa.inside(ga, gb, pairs, mode=0)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return out.cpu().numpy(), pa.inside_stats_dict(st)


def _preds(env, ga, gb, pairs, cfg=None):
    torch, pa, oracle = env
    got = {}
    for name in pa.PREDICATES:
        f, _, ist, status = pa.predicate(ga, gb, pairs, name, cfg)
        torch.cuda.synchronize()
        assert int(status.item()) == 0, name
        got[name] = f.cpu().numpy()
    return got


def _compare(env, A, B, pairs, width=4, leaf=4, check_preds=True):
    torch, pa, oracle = env
    ga, gb = _blobs(pa, A, B, width, leaf)
    bits, st = _bits(env, ga, gb, pairs)
    ref = oracle.join_predicates(A, B, pairs)
    bad = np.nonzero(bits != ref["inside_bits"])[0]
    assert bad.size == 0, (bad[:10], bits[bad[:10]], ref["inside_bits"][bad[:10]])
    if check_preds:
        got = _preds(env, ga, gb, pairs)
        for name in pa.PREDICATES:
            bad = np.nonzero(got[name] != ref[name])[0]
            assert bad.size == 0, (name, bad[:10])
    return bits, st, ref


def _hand(env):
    cases = json.load(open(os.path.join(HERE, "golden", "hand_cases.json")))["cases"]
    mk = lambda key: ci.synth.concat_meshes(  # noqa: E731
        [(np.asarray(c[key]["verts"], np.float64), np.asarray(c[key]["faces"])) for c in cases])
    return cases, mk("A"), mk("B"), np.stack([np.arange(len(cases))] * 2, 1).astype(np.int32)


@pytest.mark.parametrize("wl", [(2, 1), (4, 4), (8, 8)])
def test_hand_cases(env, wl):
    cases, A, B, pairs = _hand(env)
    bits, st, ref = _compare(env, A, B, pairs, *wl)
    # the construction facts, not only the oracle
    for k, c in enumerate(cases):
        assert ref["contains"][k] == c["contains"] and ref["within"][k] == c["within"], c["name"]
    _compare(env, B, A, pairs, *wl)


@pytest.mark.parametrize("shape", ["cube", "tet", "oct"])
def test_lattice_probes(env, shape):
    """Lattice points as representative vertices of tiny probe meshes: +z rays
    run along the solid's vertical edges, through its vertices and inside
    its face planes; points lie on faces, edges and vertices."""
    v, f, pts = {"cube": (ci.CUBE_V, ci.CUBE_F, ci.lattice(-0.5, 1.5, 0.25)),
                 "tet": (ci.TET_V, ci.TET_F, ci.lattice(-0.25, 1.25, 0.125)),
                 "oct": (ci.OCT_V, ci.OCT_F, ci.lattice(-1.25, 1.25, 0.25))}[shape]
    A = ci.mesh_set((v, f))
    B = ci.probes(pts)
    pairs = np.stack([np.zeros(B.n_meshes, np.int32), np.arange(B.n_meshes, dtype=np.int32)], 1)
    for wl in ((2, 1), (4, 4)):
        bits, st, ref = _compare(env, A, B, pairs, *wl, check_preds=wl == (4, 4))
        assert (bits & 1).sum() > 0 and (bits & 4).sum() > 0   # inside and on-surface probes exist


def test_torus_probes(env):
    rng = np.random.default_rng(12)
    v, f = ci.torus(2.0, 1.0, 24, 24)
    A = ci.mesh_set((v.astype(np.float32), f))
    pts = rng.uniform([-3.4, -3.4, -1.4], [3.4, 3.4, 1.4], size=(600, 3)).astype(np.float32)
    B = ci.probes(pts)
    pairs = np.stack([np.zeros(B.n_meshes, np.int32), np.arange(B.n_meshes, dtype=np.int32)], 1)
    bits, st, ref = _compare(env, A, B, pairs, 4, 2, check_preds=False)
    assert 50 < (bits & 1).sum() < 550


@pytest.mark.parametrize("wl", [(2, 1), (4, 4), (8, 2)])
def test_nested_grid_shapes(env, wl):
    A, B = ci.nested_grid_pairs()
    pairs = np.stack([np.arange(A.n_meshes)] * 2, 1).astype(np.int32)
    bits, st, ref = _compare(env, A, B, pairs, *wl)
    assert ref["contains"].sum() >= 10 and ref["overlap"].sum() >= 10


@pytest.mark.parametrize("wl", [(2, 1), (4, 4), (8, 8)])
def test_spheres(env, wl):
    A, B, info, tf = ci.spheres(n=300)
    pairs = np.stack([np.arange(A.n_meshes)] * 2, 1).astype(np.int32)
    bits, st, ref = _compare(env, A, B, pairs, *wl)
    assert ref["contains"].sum() >= 10 and ref["within"].sum() >= 10
    # every pair combination through the filter as well
    torch, pa, oracle = env
    ga, gb = _blobs(pa, A, B, *wl)
    cand = pa.filter_pairs(ga, gb).cpu().numpy()
    got = _preds(env, ga, gb, cand)
    ref2 = oracle.join_predicates(A, B, cand)
    for name in pa.PREDICATES:
        assert np.array_equal(got[name], ref2[name]), name


def test_predicate_matches_composed_calls(env):
    """refine_predicate equals refine + inside_pairs in the predicate's mode,
    and swapping the datasets swaps contains and within."""
    torch, pa, oracle = env
    A, B, info, tf = ci.spheres(seed=3, n=200)
    pairs = np.stack([np.arange(A.n_meshes)] * 2, 1).astype(np.int32)
    ga, gb = _blobs(pa, A, B)
    cross, _, _ = pa.refine(ga, gb, pairs)
    for name in ("contains", "within", "intersection"):
        comp, _, status = pa.inside(ga, gb, pairs, mode=name, cross=cross)
        one, _, _, _ = pa.predicate(ga, gb, pairs, name)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert np.array_equal(comp.cpu().numpy(), one.cpu().numpy()), name
    got = _preds(env, ga, gb, pairs)
    rev = _preds(env, gb, ga, pairs[:, ::-1].copy())
    assert np.array_equal(got["contains"], rev["within"]) and np.array_equal(got["within"], rev["contains"])
    assert np.array_equal(got["intersection"], rev["intersection"])


def test_deep_stack_rerun(env):
    """65,536 stacked thin boxes in one mesh (786,432 triangles): a +z column
    from below meets 262,144 leaves of a width-8, one-triangle-per-leaf tree,
    whose pending siblings exceed the fast kernel's stack, so the rays are
    rerun by the full-depth kernel; the result equals the oracle's."""
    torch, pa, oracle = env
    v, f = ci.plates(65536)
    A = ci.mesh_set((v, f))
    h = 2.0 ** -10
    pts = [[0, 0, -1], [0.25, 0.125, 10 * h + h / 2], [0.25, 0.125, 11 * h + h / 2], [0.5, -0.5, 80000 * h + h / 4]]
    B = ci.probes(pts, size=2.0 ** -14)
    pairs = np.stack([np.zeros(len(pts), np.int32), np.arange(len(pts), dtype=np.int32)], 1)
    ga, gb = _blobs(pa, A, B, 8, 1)
    bits, st = _bits(env, ga, gb, pairs)
    assert st["deep"] >= 3, st
    ref = oracle.inside_pairs(A, B, pairs)
    assert np.array_equal(bits, ref), (bits, ref)
    assert list(bits & 1) == [0, 1, 0, 1]


def test_c3_sample_full_size(env):
    """Sampled pairs of the pathology-shaped pool at full size (meshes of up
    to 100,000 triangles), every predicate against the oracle."""
    torch, pa, oracle = env
    from paper_2609_24513_amd import synth
    A, B, pairs = synth.make_c3()
    rng = np.random.default_rng(9)
    take = np.sort(rng.choice(pairs.shape[0], 96, replace=False))
    sub = pairs[take]
    ga, gb = _blobs(pa, A, B)
    got = _preds(env, ga, gb, sub)
    bits, st = _bits(env, ga, gb, sub)
    ref = oracle.join_predicates(A, B, sub)
    free = ref["overlap"] == 0
    assert np.array_equal(bits[free], ref["inside_bits"][free])
    for name in pa.PREDICATES:
        assert np.array_equal(got[name], ref[name]), name
    # the whole candidate list runs; the intersection join is a superset of overlap
    full = _preds(env, ga, gb, pairs)
    assert np.all(full["intersection"] >= full["overlap"])
    assert not np.any(full["contains"] & full["overlap"]) and not np.any(full["within"] & full["overlap"])
    assert np.array_equal(full["intersection"], full["overlap"] | full["contains"] | full["within"])


def test_empty_and_errors(env):
    torch, pa, oracle = env
    cases, A, B, pairs = _hand(env)
    ga, gb = _blobs(pa, A, B)
    out, st, status = pa.inside(ga, gb, pairs[:0], mode=0)
    f, _, _, status2 = pa.predicate(ga, gb, pairs[:0], "contains")
    torch.cuda.synchronize()
    assert out.numel() == 0 and f.numel() == 0 and int(status.item()) == 0 and int(status2.item()) == 0
    bad = np.array([[0, 0], [len(cases), 0], [0, -1]], np.int32)
    out, st, status = pa.inside(ga, gb, bad, mode=0)
    torch.cuda.synchronize()
    assert int(status.item()) == -1
    lib = pa._lib.load()
    assert lib.inside_pairs(ga.ptr, ga.n_meshes, gb.ptr, gb.n_meshes, None, 1, 0, None, None, None, None, None, 0,
                            None) == pa._lib.PR_E_ARG
    with pytest.raises(pa.PierceError):
        pa.inside(ga, gb, pairs, mode=5, cross=np.zeros(len(cases), np.uint8))
    with pytest.raises(ValueError):
        pa.inside(ga, gb, pairs, mode=1)
