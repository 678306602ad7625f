"""Serving (continuous batching) on the GPU: every request's answer is the same
when it runs alone and when it is served in the mix, with a normal and with a
zero HBM budget (requests queue, none is dropped); a sample is checked
against the exact CPU oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool():
    import torch
    assert torch.cuda.is_available()
    import paper_2609_24513_amd as pa
    from paper_2609_24513_amd import synth
    R, S = synth.make_c5_pool(n_meshes=6000, side=29.0)
    gr, gs = pa.MeshBlob.build(R), pa.MeshBlob.build(S)
    return R, S, gr, gs


@pytest.mark.parametrize("budget", [1 << 30, 0])
def test_served_equals_alone(pool, budget):
    from paper_2609_24513_amd import serve
    R, S, gr, gs = pool
    trace = serve.make_trace(R.aabbs(), S.aabbs(), 80, lam=3000.0, seed=11, k_hi=1500.0, space=29.0)
    srv = serve.JoinServer(gr, gs, max_req_per_batch=8, slots=3, hbm_budget=budget)
    out = srv.run(trace)
    assert all(r.t_done >= r.t_arrival for r in out)
    assert srv.batches >= 2
    n_pairs = 0
    for r in out:
        pairs, flags = srv.query_alone(r.box)
        assert np.array_equal(r.pairs, pairs), r.rid
        assert np.array_equal(r.flags, flags), r.rid
        n_pairs += pairs.shape[0]
    assert n_pairs > 100


def test_served_sample_against_oracle(pool):
    import oracle
    from paper_2609_24513_amd import serve
    R, S, gr, gs = pool
    trace = serve.make_trace(R.aabbs(), S.aabbs(), 30, lam=2000.0, seed=12, k_hi=800.0, space=29.0)
    out = serve.JoinServer(gr, gs, max_req_per_batch=8, slots=2).run(trace)
    for r in out[:10]:
        if r.pairs.shape[0]:
            want = oracle.join(R, S, r.pairs, mode=1)
            assert np.array_equal(r.flags, want), r.rid


def test_plain_path_same_results(pool):
    from paper_2609_24513_amd import serve
    R, S, gr, gs = pool
    trace = serve.make_trace(R.aabbs(), S.aabbs(), 12, lam=500.0, seed=13, k_hi=300.0, space=29.0)
    a = serve.JoinServer(gr, gs, max_req_per_batch=4, slots=2).run(
        [serve.Request(r.rid, r.t_arrival, r.box) for r in trace])
    b = serve.run_plain(gr, gs, trace)
    for x, y in zip(a, b):
        assert np.array_equal(x.pairs, y.pairs) and np.array_equal(x.flags, y.flags)
