"""GPU parity of the paper's dataset-level overlap join (one BVH over every
triangle of a dataset, all hits of every edge, Sections 3.2 and 3.5) and of
the selectivity estimate, through the C ABI.

The joined pair set of every materialisation strategy (counting two-pass,
estimated hashmap, fixed hashmap with forced regrowth) equals the oracle's:
every closed-box candidate pair the exact oracle finds intersecting.  The
estimate equals the oracle's step-by-step evaluation up to the order of
FP64 summation.
"""
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
    from paper_2609_24513_amd import dataset as ds, synth
    return torch, pa, ds, synth, oracle


def _workload(synth, name):
    if name == "c1":
        return synth.make_c1()
    if name == "sweep1":
        return synth.make_sweep(1)
    if name == "c2small":
        return synth.make_c2(n_nuclei=1000, n_vessels=100, box=464.0)
    A, B, info, tf = ci.spheres(seed=5, n=200)
    return A, B


def _oracle_set(oracle, A, B):
    cand = oracle.candidate_pairs(oracle.mesh_boxes(A), oracle.mesh_boxes(B))
    return cand[oracle.join(A, B, cand) == 1]


@pytest.mark.parametrize("name,w,l", [("c1", 4, 4), ("sweep1", 8, 2), ("spheres", 4, 2), ("c2small", 8, 2)])
def test_dataset_join_all_strategies(env, name, w, l):
    torch, pa, ds, synth, oracle = env
    A, B = _workload(synth, name)
    want = _oracle_set(oracle, A, B)
    ga, gb = pa.MeshBlob.build(A, width=w, leaf_size=l), pa.MeshBlob.build(B, width=w, leaf_size=l)
    da, db = ds.DatasetBlob.build(A, width=w, leaf_size=l), ds.DatasetBlob.build(B, width=w, leaf_size=l)
    ma, mb = ds.max_groups(A), ds.max_groups(B)
    results = {}
    for strat, kw in (("two_pass", {}), ("estimated", {}), ("fixed", {"fixed_slots": 4})):
        got, info = ds.join_dataset(ga, gb, da, db, ma, mb, strategy=strat, **kw)
        assert np.array_equal(got, want), (strat, got.shape, want.shape)
        results[strat] = info
    assert results["two_pass"]["records"] >= want.shape[0]
    if want.shape[0] > 4:
        assert results["fixed"]["relaunches"] >= 1
    # the per-pair path gives the same set
    cand = pa.filter_pairs(ga, gb)
    flags, _, _ = pa.refine(ga, gb, cand, pa.RefineConfig(schedule=1))
    torch.cuda.synchronize()
    assert np.array_equal(cand.cpu().numpy()[flags.cpu().numpy() == 1], want)


@pytest.mark.parametrize("name,cells", [("c1", 4), ("sweep1", 16), ("c2small", 32), ("spheres", 8)])
def test_estimate_matches_oracle(env, name, cells):
    torch, pa, ds, synth, oracle = env
    A, B = _workload(synth, name)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    got = ds.estimate(ga, gb, cells)
    want = oracle.estimate.estimate(A, B, oracle.mesh_boxes(A), oracle.mesh_boxes(B), cells)["estimate"]
    assert want > 0
    assert got == pytest.approx(want, rel=1e-9, abs=1e-9)


def test_dataset_errors(env):
    torch, pa, ds, synth, oracle = env
    A, B = synth.make_c1(n=3)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    da = ds.DatasetBlob.build(A)
    # a per-mesh blob of several meshes is not a dataset-level target
    tr = ds._Tracer(gb, ds.max_groups(B), ds.DatasetBlob(ga, da.tri_obj, A.n_meshes, da.f_total), 1)
    tr.run(0)
    torch.cuda.synchronize()
    assert int(tr.status.item()) == pa._lib.PR_E_UNSUPPORTED
    # too few groups declared for the source
    tr = ds._Tracer(gb, 1, da, 1)
    tr.run(0)
    torch.cuda.synchronize()
    assert int(tr.status.item()) == pa._lib.PR_E_UNSUPPORTED
