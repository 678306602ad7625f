"""Serving (continuous batching) on the GPU.

* Every request's answer is the same when it runs alone and when it is
  served in the mix, with a normal and with a zero HBM budget (requests
  queue, none is dropped).
* On the full serving pool (50,000 resident level-2 icospheres in a
  58.5^3 box, split by id parity), every served request of a seeded trace
  with query boxes selecting up to 5,000 candidate pairs, served 32 to a
  batch, is checked against the oracle: its candidate pairs against the
  closed-box definition with its query box, its flags against the exact
  join.
* A request selecting more candidates than a batch region holds is
  answered in full (on its own), not truncated.
"""
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
    # the budget is spent on slots: as many as it holds, at least one
    assert len(srv.slots) == max(1, min(3, budget // srv.slot_bytes))
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


def _check_against_oracle(R, S, out):
    import oracle
    br, bs = oracle.mesh_boxes(R), oracle.mesh_boxes(S)
    allp, allf = [], []
    for r in out:
        want = oracle.candidate_pairs(br, bs, r.box)
        assert np.array_equal(r.pairs, want), r.rid
        allp.append(r.pairs)
        allf.append(r.flags)
    allp = np.concatenate(allp).astype(np.int32)
    allf = np.concatenate(allf)
    want = oracle.join(R, S, allp, mode=1)
    assert np.array_equal(allf, want), np.nonzero(allf != want)[0][:10]
    return allp.shape[0], int(want.sum())


def test_served_sample_against_oracle(pool):
    from paper_2609_24513_amd import serve
    R, S, gr, gs = pool
    trace = serve.make_trace(R.aabbs(), S.aabbs(), 30, lam=2000.0, seed=12, k_hi=800.0, space=29.0)
    out = serve.JoinServer(gr, gs, max_req_per_batch=8, slots=2).run(trace)
    n, t = _check_against_oracle(R, S, out)
    assert n > 100 and t > 10


def test_full_pool_every_request_against_oracle():
    """The serving workload at full size: 50,000 meshes, queries of up to
    5,000 candidate pairs, batches of 32 requests (closed loop, so batches
    are full and requests mix on the device), then a real-time stretch."""
    import torch
    import paper_2609_24513_amd as pa
    from paper_2609_24513_amd import serve, synth
    R, S = synth.make_c5_pool()
    assert R.n_meshes + S.n_meshes == 50_000
    gr, gs = pa.MeshBlob.build(R), pa.MeshBlob.build(S)
    br, bs = R.aabbs(), S.aabbs()
    trace = serve.make_trace(br, bs, 96, lam=1000.0, seed=21)
    srv = serve.JoinServer(gr, gs, max_req_per_batch=32, slots=3)
    out = srv.run(trace, realtime=False)
    assert srv.batches <= 6 and srv.oversized == 0
    assert max(r.pairs.shape[0] for r in out) > 2000
    n, t = _check_against_oracle(R, S, out)
    assert n > 20_000 and t > 1000
    trace2 = serve.make_trace(br, bs, 64, lam=1000.0, seed=22)
    out2 = serve.JoinServer(gr, gs, max_req_per_batch=32, slots=3).run(trace2, realtime=True)
    _check_against_oracle(R, S, out2)
    del gr, gs
    torch.cuda.empty_cache()


def test_oversized_request_not_truncated(pool):
    """Query boxes selecting more candidates than max_pairs: the answer is
    the whole join, equal to the request alone and to the oracle."""
    from paper_2609_24513_amd import serve
    R, S, gr, gs = pool
    trace = serve.make_trace(R.aabbs(), S.aabbs(), 24, lam=2000.0, seed=14, k_lo=100.0, k_hi=3000.0,
                             space=29.0, min_pairs=1, max_pairs=2500)
    srv = serve.JoinServer(gr, gs, max_req_per_batch=8, slots=2, max_pairs=400)
    out = srv.run(trace)
    assert srv.oversized > 0
    assert max(r.pairs.shape[0] for r in out) > 400
    for r in out:
        pairs, flags = srv.query_alone(r.box)
        assert np.array_equal(r.pairs, pairs) and np.array_equal(r.flags, flags), r.rid
    _check_against_oracle(R, S, out)


def test_graph_batches_match_eager(pool):
    """Batches replayed from the captured graphs (several replays of each
    batch size, with the loop's own host work and synchronisations between
    them) against the same trace served eagerly, request by request, and
    against the oracle."""
    from paper_2609_24513_amd import serve
    R, S, gr, gs = pool
    trace = serve.make_trace(R.aabbs(), S.aabbs(), 40, lam=2000.0, seed=15, k_hi=800.0, space=29.0)
    g = serve.JoinServer(gr, gs, max_req_per_batch=4, slots=2)
    assert g.graphs and all(len(s.graphs) == 4 for s in g.slots)
    a = g.run([serve.Request(r.rid, r.t_arrival, r.box) for r in trace], realtime=False)
    assert g.batches >= 10
    e = serve.JoinServer(gr, gs, max_req_per_batch=4, slots=2, graphs=False)
    assert not e.graphs
    b = e.run([serve.Request(r.rid, r.t_arrival, r.box) for r in trace], realtime=False)
    for x, y in zip(a, b):
        assert x.rid == y.rid
        assert np.array_equal(x.pairs, y.pairs) and np.array_equal(x.flags, y.flags), x.rid
    _check_against_oracle(R, S, a)


def test_plain_path_same_results(pool):
    from paper_2609_24513_amd import serve
    R, S, gr, gs = pool
    trace = serve.make_trace(R.aabbs(), S.aabbs(), 12, lam=500.0, seed=13, k_hi=300.0, space=29.0)
    a = serve.JoinServer(gr, gs, max_req_per_batch=4, slots=2).run(
        [serve.Request(r.rid, r.t_arrival, r.box) for r in trace])
    b = serve.run_plain(gr, gs, trace)
    for x, y in zip(a, b):
        assert np.array_equal(x.pairs, y.pairs) and np.array_equal(x.flags, y.flags)
