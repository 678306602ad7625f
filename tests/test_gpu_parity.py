"""GPU parity: the HIP path (through the C ABI) against the exact CPU oracle.

Flags are compared bit for bit (the predicate has exactly one correct answer
per pair).  Cases: hand-built contact cases, the tiny config (all pairs), a
precision-stress sample on a 2^-10 grid, a scaled pathology-shaped config,
every BVH width / leaf size / launch form / precision mode, queue overflow,
coordinates outside the FP32-safe range, and argument/geometry errors.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import oracle
    oracle.build(force=False)
    import paper_2609_24513_amd as pa
    from paper_2609_24513_amd import synth
    return torch, pa, synth, oracle


def _hand(synth):
    cases = json.load(open(os.path.join(HERE, "golden", "hand_cases.json")))["cases"]
    A = synth.concat_meshes([(np.asarray(c["A"]["verts"], np.float64), np.asarray(c["A"]["faces"])) for c in cases])
    B = synth.concat_meshes([(np.asarray(c["B"]["verts"], np.float64), np.asarray(c["B"]["faces"])) for c in cases])
    pairs = np.stack([np.arange(len(cases))] * 2, 1).astype(np.int32)
    exp = np.array([c["expected"] for c in cases], np.uint8)
    return A, B, pairs, exp


def _run(env, A, B, pairs, width=4, leaf=4, builder=0, **cfg):
    torch, pa, synth, oracle = env
    ga = pa.MeshBlob.build(A, width=width, leaf_size=leaf, builder=builder)
    gb = pa.MeshBlob.build(B, width=width, leaf_size=leaf, builder=builder)
    flags, stats, status = pa.refine(ga, gb, pairs, pa.RefineConfig(**cfg))
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return flags.cpu().numpy(), pa.stats_dict(stats)


CONFIGS = [dict(width=w, leaf=l, persistent=p, precision=q, schedule=sc, builder=(w + l + q) % 2)
           for w in (2, 4, 8) for l in (1, 4, 8) for p in (0, 1) for q in (0, 1, 2, 3) for sc in (0, 1, 2)
           if not (l == 8 and q == 1) and not (p == 0 and sc != 1)]


@pytest.mark.parametrize("c", CONFIGS, ids=lambda c: "w%d_l%d_p%d_q%d_s%d_b%d" % (
    c["width"], c["leaf"], c["persistent"], c["precision"], c["schedule"], c["builder"]))
def test_hand_cases_all_configs(env, c):
    torch, pa, synth, oracle = env
    A, B, pairs, exp = _hand(synth)
    got, st = _run(env, A, B, pairs, **c)
    assert np.array_equal(got, exp), [i for i in np.nonzero(got != exp)[0]]
    # roles swapped
    got2, _ = _run(env, B, A, pairs, **c)
    assert np.array_equal(got2, exp)


def test_build_metadata_c1(env):
    torch, pa, synth, oracle = env
    A, B = synth.make_c1()
    ga = pa.MeshBlob.build(A)
    assert np.array_equal(ga.boxes().cpu().numpy(), oracle.mesh_boxes(A))
    ec = ga.edge_counts().cpu().numpy()
    for m in range(A.n_meshes):
        v, f = A.mesh(m)
        assert ec[m] == oracle.unique_edges(f).shape[0]


def _blob_nodes(blob, W):
    """(mesh descriptors, node child ids) read back from a blob's bytes."""
    b = blob.blob.cpu().numpy().view(np.uint8)
    h = b[:256]
    n_meshes, off_mesh, off_node = (int(np.frombuffer(h[o:o + 8].tobytes(), np.int64)[0]) for o in (16, 56, 64))
    desc = np.frombuffer(b[off_mesh:off_mesh + 64 * n_meshes].tobytes(), np.int32).reshape(n_meshes, 16)
    n_nodes = int((desc[:, 6] + desc[:, 7]).max())
    node = np.frombuffer(b[off_node:off_node + 32 * W * n_nodes].tobytes(), np.int32).reshape(n_nodes, 8 * W)
    return desc, node[:, 6 * W:7 * W]


def test_root_children_follow_root(env):
    """Layout the cull relies on: a root's internal children are the nodes
    right after it, in child order (so the second level is addressed from
    the root's index alone)."""
    torch, pa, synth, oracle = env
    A, _ = synth.make_c1()
    big = synth.concat_meshes([synth.icosphere(k) for k in (0, 1, 2, 3, 4, 5)])
    for S in (A, big):
        for W in (2, 4, 8):
            for L, builder in ((1, 0), (4, 1), (8, 0)):
                g = pa.MeshBlob.build(S, width=W, leaf_size=L, builder=builder)
                desc, child = _blob_nodes(g, W)
                for m in range(S.n_meshes):
                    root, n = int(desc[m, 14]), int(desc[m, 7])
                    if n == 0:
                        continue
                    inner = [int(c) for c in child[root] if 0 <= c < 0x7fffffff]
                    assert inner == list(range(root + 1, root + 1 + len(inner))), (W, L, m)
                    assert len(inner) <= n - 1


def _exp_range_np(S):
    """(lowest, highest) set-bit exponent over the coordinates of every face."""
    v = S.verts.astype(np.float32)
    used = np.concatenate([S.vert_off[m] + S.faces[S.face_off[m]:S.face_off[m + 1]].reshape(-1)
                           for m in range(S.n_meshes)])
    x = np.abs(v[np.unique(used)].reshape(-1).astype(np.float64))
    x = x[x > 0]
    hi = np.floor(np.log2(x)).astype(int)
    lo = hi.copy()
    for k in range(x.shape[0]):        # lowest set bit: largest e with x / 2^e an integer
        e = hi[k] - 23
        while np.ldexp(x[k], -(e + 1)) == np.floor(np.ldexp(x[k], -(e + 1))):
            e += 1
        lo[k] = e
    return int(lo.min()), int(hi.max())


def test_coord_exponent_range(env):
    """The build records the coordinates' bit-exponent range; the precision-
    stress pairs (2^-10 grid, radius ~1) qualify for the in-place grid tier,
    the tiny config's random coordinates do not."""
    torch, pa, synth, oracle = env
    A, B, pairs, _ = synth.make_c4(n_pairs=20)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    assert ga.exp_range() == _exp_range_np(A) and gb.exp_range() == _exp_range_np(B)
    assert pa.small_grid(ga, gb)
    A1, B1 = synth.make_c1(n=3)
    g1 = pa.MeshBlob.build(A1)
    assert g1.exp_range() == _exp_range_np(A1)
    assert not pa.small_grid(g1, pa.MeshBlob.build(B1))


def test_filter_matches_exact_boxes(env):
    torch, pa, synth, oracle = env
    for seed in (1, 2, 3):
        A, B = synth.make_c1(seed=seed, n=20)
        ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
        got = pa.filter_pairs(ga, gb).cpu().numpy()
        assert np.array_equal(got, oracle.candidate_pairs(oracle.mesh_boxes(A), oracle.mesh_boxes(B)))


def _tetra_set(synth, n, seed, side):
    """n small random tetrahedra (4 faces each) scattered in [0, side]^3."""
    rng = np.random.default_rng(seed)
    tf = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], np.int32)
    c = rng.uniform(0, side, size=(n, 1, 3))
    v = (c + rng.uniform(-0.5, 0.5, size=(n, 4, 3))).astype(np.float32).reshape(-1, 3)
    f = np.tile(tf, (n, 1))
    off4 = np.arange(n + 1, dtype=np.int64) * 4
    return synth.MeshSet(v, f, off4, off4.copy())


@pytest.mark.parametrize("na,nb", [(300, 70_000), (70_000, 50)])
def test_filter_large_mesh_counts(env, na, nb):
    """Datasets above the single-block scan limit take the device-scan path
    for the kept lists and the row offsets."""
    torch, pa, synth, oracle = env
    A, B = _tetra_set(synth, na, 11, 30.0), _tetra_set(synth, nb, 12, 30.0)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    got = pa.filter_pairs(ga, gb).cpu().numpy()
    assert np.array_equal(got, oracle.candidate_pairs(oracle.mesh_boxes(A), oracle.mesh_boxes(B)))


def _tetra_set_with_empties(synth, n, seed, side, every=7):
    """Like _tetra_set, with every `every`-th mesh empty (no vertices, no faces)."""
    full = _tetra_set(synth, n, seed, side)
    keep = np.arange(n) % every != 3
    v = full.verts.reshape(n, 4, 3)[keep].reshape(-1, 3)
    f = full.faces.reshape(n, 4, 3)[keep].reshape(-1, 3)
    sizes = np.where(keep, 4, 0)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return synth.MeshSet(v, f, off, off.copy())


@pytest.mark.parametrize("na,nb", [(1, 1), (17, 4096), (65_536, 4_097), (65_537, 300), (131_072, 40), (131_073, 30),
                                   (500, 4_097)])
def test_filter_row_block_path_limits(env, na, nb):
    """Row and column counts on both sides of the limits of the 64-rows-per-block
    path (4,096 columns, 131,072 rows; with a query box 65,536 rows), with empty
    meshes mixed in, with and without a query box, and a capacity below the count."""
    torch, pa, synth, oracle = env
    A = _tetra_set_with_empties(synth, na, 21, 30.0)
    B = _tetra_set_with_empties(synth, nb, 22, 30.0)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    ba, bb = oracle.mesh_boxes(A), oracle.mesh_boxes(B)
    want = oracle.candidate_pairs(ba, bb)
    got = pa.filter_pairs(ga, gb).cpu().numpy()
    assert np.array_equal(got, want)
    q = np.array([5, 2, 4, 22, 25, 19], np.float32)
    got = pa.filter_pairs(ga, gb, query_box=q).cpu().numpy()
    assert np.array_equal(got, oracle.candidate_pairs(ba, bb, q))
    if want.shape[0] > 1:
        cap = want.shape[0] // 2
        buf, cnt = pa.filter_pairs(ga, gb, cap=cap, sync=False)
        assert int(cnt.item()) == want.shape[0]
        assert np.array_equal(buf[:cap].cpu().numpy(), want[:cap])


@pytest.mark.parametrize("n_regions,region_cap,cap", [(0, 10, 5), (1, 7, 7), (5, 100, 1000), (32, 5000, 40_000),
                                                        (300, 3, 2000)])
def test_gather_regions_matches_numpy(env, n_regions, region_cap, cap):
    """Region concatenation with counts on the device: counts below, at and
    above the region size (clamped), negative counts (none), and an output
    smaller than the total (rows dropped, exact total still reported)."""
    torch, pa, synth, oracle = env
    rng = np.random.default_rng(n_regions * 7 + region_cap)
    regions = rng.integers(-5, 1 << 20, size=(max(n_regions, 1) * region_cap, 2)).astype(np.int32)
    counts = rng.integers(-2, region_cap + 3, size=max(n_regions, 1)).astype(np.int64)[:n_regions]
    keep = [regions[k * region_cap:k * region_cap + min(max(c, 0), region_cap)] for k, c in enumerate(counts)]
    want = np.concatenate(keep) if keep else np.zeros((0, 2), np.int32)
    out = torch.full((cap, 2), -7, dtype=torch.int32, device="cuda")
    total = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    pa.gather_regions(torch.as_tensor(regions).cuda(), region_cap,
                      torch.as_tensor(counts if n_regions else np.zeros(1, np.int64)).cuda(), n_regions, out, total)
    torch.cuda.synchronize()
    assert int(total.item()) == want.shape[0]
    m = min(cap, want.shape[0])
    got = out.cpu().numpy()
    assert np.array_equal(got[:m], want[:m])
    assert (got[m:] == -7).all()


@pytest.mark.parametrize("n", [1, 4096, 65_536, 100_003])
def test_compact_matches_numpy(env, n):
    """Ordered compaction on both sides of the single-block limit."""
    torch, pa, synth, oracle = env
    rng = np.random.default_rng(n)
    pairs = rng.integers(0, 1 << 20, size=(n, 2)).astype(np.int32)
    flags = (rng.random(n) < 0.3).astype(np.uint8)
    got = pa.compact(torch.as_tensor(pairs).cuda(), torch.as_tensor(flags).cuda()).cpu().numpy()
    assert np.array_equal(got, pairs[flags == 1])


@pytest.mark.parametrize("n", [5_000, 65_536, 100_003])
def test_compact_device_count_and_capacity(env, n):
    """Compaction through the C ABI with a device pair count below n and an
    output capacity below the flagged count: the first cap flagged pairs
    (in input order) are written and the exact count is reported."""
    import ctypes
    from paper_2609_24513_amd import _lib
    torch, pa, synth, oracle = env
    rng = np.random.default_rng(n + 1)
    pairs = rng.integers(0, 1 << 20, size=(n, 2)).astype(np.int32)
    flags = (rng.random(n) < 0.4).astype(np.uint8)
    live = n - n // 7
    want = pairs[:live][flags[:live] == 1]
    cap = want.shape[0] // 2
    lib = _lib.load()
    wb = ctypes.c_size_t(0)
    _lib.check(lib.compact_pairs_ws_bytes(n, ctypes.byref(wb)))
    ws = torch.empty(max(256, wb.value), dtype=torch.uint8, device="cuda")
    p_d, f_d = torch.as_tensor(pairs).cuda(), torch.as_tensor(flags).cuda()
    nd = torch.tensor([live], dtype=torch.int64, device="cuda")
    out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    _lib.check(lib.compact_pairs(p_d.data_ptr(), f_d.data_ptr(), n, nd.data_ptr(), out.data_ptr(), cap,
                                 cnt.data_ptr(), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert int(cnt.item()) == want.shape[0]
    assert np.array_equal(out.cpu().numpy(), want[:cap])


def test_filter_query_box_and_capacity(env):
    torch, pa, synth, oracle = env
    A, B = synth.make_c1(seed=4, n=40)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    rng = np.random.default_rng(0)
    for _ in range(10):
        c = rng.uniform(0, 4, size=3); h = rng.uniform(0.2, 2.0, size=3)
        q = np.concatenate([c - h, c + h]).astype(np.float32)
        got = pa.filter_pairs(ga, gb, query_box=q).cpu().numpy()
        assert np.array_equal(got, oracle.candidate_pairs(oracle.mesh_boxes(A), oracle.mesh_boxes(B), q))
    full = oracle.candidate_pairs(oracle.mesh_boxes(A), oracle.mesh_boxes(B))
    got = pa.filter_pairs(ga, gb, cap=3).cpu().numpy()  # relaunch path
    assert np.array_equal(got, full)


def test_c1_all_pairs_against_oracle(env):
    torch, pa, synth, oracle = env
    A, B = synth.make_c1()
    pairs = np.array([(i, j) for i in range(8) for j in range(8)], np.int32)
    want = oracle.join(A, B, pairs, mode=0)
    for w, l in ((2, 1), (4, 4), (8, 8)):
        for p in (0, 1):
            got, st = _run(env, A, B, pairs, width=w, leaf=l, persistent=p, precision=0)
            assert np.array_equal(got, want), (w, l, p)
            assert st["pairs_true"] == int(want.sum())


def test_c4_precision_stress_sample(env):
    torch, pa, synth, oracle = env
    A, B, pairs, cls = synth.make_c4(n_pairs=240)
    want = oracle.join(A, B, pairs, mode=1)
    results = {}
    for q in (0, 1, 2):
        for p in (0, 1):
            got, st = _run(env, A, B, pairs, persistent=p, precision=q)
            assert np.array_equal(got, want), (q, p, np.nonzero(got != want)[0][:10])
            results[(q, p)] = st
    assert results[(0, 1)]["fp32_ambiguous"] > 0
    assert results[(0, 1)]["exact_decided"] > 0


def test_c4_full_precision_stress_zero_mismatches(env):
    """All 2,000 pairs of the precision-stress config, both launch forms."""
    torch, pa, synth, oracle = env
    A, B, pairs, cls = synth.make_c4()
    want = oracle.join(A, B, pairs, mode=1)
    for p in (1, 0):
        got, st = _run(env, A, B, pairs, persistent=p, precision=0)
        assert int((got != want).sum()) == 0, (p, np.nonzero(got != want)[0][:10])
        assert st["fp32_ambiguous"] > 0 and st["exact_decided"] > 0
    contact = np.array([c != "random" for c in cls])
    assert want[contact].all()


def test_c3_scaled_all_widths_and_schedules(env):
    """Batching-shaped pairs (face counts log-uniform in [500, 20,000]) for every
    width, leaf size and schedule; also a tiny work-item size."""
    torch, pa, synth, oracle = env
    A, B, pairs = synth.make_c3(n_pairs=3000, n_pool=256, f_hi=20000.0)
    want = oracle.join(A, B, pairs, mode=1)
    assert 0 < want.sum() < pairs.shape[0]
    for w in (2, 4, 8):
        for l in (1, 2, 4, 8):
            bld = (w // 2 + l) % 2
            ga = pa.MeshBlob.build(A, width=w, leaf_size=l, builder=bld)
            gb = pa.MeshBlob.build(B, width=w, leaf_size=l, builder=bld)
            for cfg in (dict(schedule=0), dict(schedule=1), dict(schedule=2), dict(schedule=0, seg_live_max=0x40201008),
                        dict(schedule=2, survivor_cap=50), dict(schedule=1, survivor_cap=50),
                        dict(schedule=1, survivor_cap=8), dict(schedule=1, grid_blocks=5),
                        dict(schedule=2, grid_blocks=100), dict(schedule=1, trace_budget=1),
                        dict(schedule=1, trace_budget=3, grid_blocks=7), dict(schedule=1, trace_budget=-1),
                        dict(schedule=1, grid_blocks=1), dict(schedule=0, grid_blocks=2, survivor_cap=50),
                        dict(schedule=1, lds_stack=1), dict(schedule=0, lds_stack=1, grid_blocks=3),
                        dict(schedule=1, precision=3), dict(schedule=2, precision=1)):
                flags, stats, status = pa.refine(ga, gb, pairs, pa.RefineConfig(persistent=1, **cfg))
                torch.cuda.synchronize()
                assert int(status.item()) == 0
                assert np.array_equal(flags.cpu().numpy(), want), (w, l, cfg)


def test_many_units_per_wave_cull(env):
    """60,000 pairs (120,000 units, more than eight per culling wave even
    with every CU at its maximum of 32 waves), so that the culling waves take
    their units a few at a time from per-XCD shares in cost order: every
    box-overlapping tetrahedron pair, mixed with random pairs and repeats,
    against the oracle in FP32-filter and exact modes."""
    torch, pa, synth, oracle = env
    assert 2 * 60_000 > 8 * 32 * torch.cuda.get_device_properties(0).multi_processor_count
    A, B = _tetra_set(synth, 600, 31, 6.0), _tetra_set(synth, 600, 32, 6.0)
    cand = oracle.candidate_pairs(oracle.mesh_boxes(A), oracle.mesh_boxes(B)).astype(np.int32)
    rng = np.random.default_rng(3)
    extra = rng.integers(0, 600, size=(60_000 - cand.shape[0], 2)).astype(np.int32)
    pairs = np.concatenate([cand, extra])[rng.permutation(60_000)]
    want = oracle.join(A, B, pairs, mode=1)
    assert 0 < want.sum() < pairs.shape[0]
    for prec in (0, 1):
        got, _ = _run(env, A, B, pairs, persistent=1, schedule=1, precision=prec)
        assert np.array_equal(got, want), prec


def test_block_sharing_matches_unshared(env):
    """Schedule 3 with the waves of a block sharing pending stack entries (the
    default) against sharing off (trace_budget=-1) and the oracle, on the
    precision-stress pairs (long exact traversals) with one and two blocks,
    where three of every four waves spend most of the run helping."""
    torch, pa, synth, oracle = env
    A, B, pairs, _ = synth.make_c4(n_pairs=300)
    want = oracle.join(A, B, pairs, mode=1)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    for cfg in (dict(grid_blocks=1), dict(grid_blocks=2), dict(), dict(trace_budget=-1, grid_blocks=1)):
        for prec in (0, 1):
            flags, stats, status = pa.refine(ga, gb, pairs, pa.RefineConfig(persistent=1, schedule=1, precision=prec,
                                                                            **cfg))
            torch.cuda.synchronize()
            assert int(status.item()) == 0, (cfg, prec)
            assert np.array_equal(flags.cpu().numpy(), want), (cfg, prec)


@pytest.mark.parametrize("schedule", [0, 1, 2])
def test_device_pair_count(env, schedule):
    """Filter -> refine -> compaction with the pair count left on the device:
    rows past the count are invalid padding that must be ignored, and the
    result equals the host-count run and the oracle."""
    torch, pa, synth, oracle = env
    A, B = synth.make_c1(seed=5, n=24)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    ref = pa.filter_pairs(ga, gb)
    n = int(ref.shape[0])
    buf, cnt = pa.filter_pairs(ga, gb, cap=n + 37, sync=False)
    buf[n:] = -7  # out-of-range ids: processing them would raise PR_E_ARG
    flags, _, status = pa.refine(ga, gb, buf, pa.RefineConfig(schedule=schedule, n_dev=cnt))
    torch.cuda.synchronize()
    assert int(cnt.item()) == n and int(status.item()) == 0
    want, _ = _run(env, A, B, ref.cpu().numpy(), schedule=schedule)
    assert np.array_equal(flags[:n].cpu().numpy(), want)
    exp = oracle.join(A, B, ref.cpu().numpy().astype(np.int64))
    assert np.array_equal(want, np.asarray(exp, np.uint8))
    res, rcnt = pa.compact(buf, flags, n_dev=cnt, sync=False)
    got = res[:int(rcnt.item())].cpu().numpy()
    assert np.array_equal(got, ref.cpu().numpy()[want == 1])


def test_autotune_small(env):
    torch, pa, synth, oracle = env
    from paper_2609_24513_amd import autotune
    A, B, pairs = synth.make_c3(n_pairs=1500, n_pool=128, f_hi=8000.0)
    res = autotune.tune(A, B, pairs, widths=(2, 4), leaves=(1, 4), schedules=(0, 1, 2), frac=0.2, reps=2,
                        use_cache=False)
    # per (width, leaf): wave-per-pair, wave-per-segment and the automatic schedule with two tables
    assert len(res["table"]) == 2 * 2 * 4
    assert sorted({(r["schedule"], r["seg_live_max"] != 0) for r in res["table"]}) == [(0, True), (1, False), (2, False)]
    b = res["best"]
    assert b["ms"] == min(r["ms"] for r in res["table"])
    assert res["per_bucket"]
    want = oracle.join(A, B, pairs, mode=1)
    got, _ = _run(env, A, B, pairs, width=b["width"], leaf=b["leaf_size"], persistent=1, schedule=b["schedule"],
                  seg_live_max=b["seg_live_max"])
    assert np.array_equal(got, want)


def test_c2_full_size_against_oracle(env):
    """The pathology-shaped workload at full size, in the launch configuration
    the benchmark times (persistent, W=4, L=4): every candidate pair."""
    torch, pa, synth, oracle = env
    A, B = synth.make_c2()
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    pairs = pa.filter_pairs(ga, gb)
    hp = pairs.cpu().numpy()
    assert np.array_equal(hp, oracle.candidate_pairs(oracle.mesh_boxes(A), oracle.mesh_boxes(B)))
    want = oracle.join(A, B, hp, mode=1)
    flags, stats, status = pa.refine(ga, gb, pairs, pa.RefineConfig(persistent=1))
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert int((flags.cpu().numpy() != want).sum()) == 0


def _c3_expected(A, B, pairs):
    """The oracle's flags for the full batching workload, stored by
    tests/golden/make_expected_flags.py (which calls only the oracle); the
    input digest must match the inputs generated here."""
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_expected_flags as mef
    digest, want = mef.load()
    assert digest == mef.input_digest(A, B, pairs), "inputs changed: rerun tests/golden/make_expected_flags.py"
    return want


def test_c3_full_size_against_oracle(env):
    """The batching workload at full size (50,000 pairs, faces up to 100,000
    per mesh), one persistent launch per configuration: first the one the
    benchmark times (W = 8, L = 1, wave-per-pair, with the cull order and the
    per-XCD grabs that 100,000 units take), then every schedule and builder at
    W = 4, L = 4; every pair checked."""
    torch, pa, synth, oracle = env
    A, B, pairs = synth.make_c3()
    want = _c3_expected(A, B, pairs)
    assert want.shape[0] == 50_000 and 0 < want.sum() < 50_000
    for w, lf, sc, bld in ((8, 1, 1, 0), (4, 4, 1, 0), (4, 4, 2, 0), (4, 4, 0, 0), (4, 4, 1, 1)):
        got, st = _run(env, A, B, pairs, width=w, leaf=lf, persistent=1, schedule=sc, builder=bld)
        assert int((got != want).sum()) == 0, (w, lf, sc, bld)
        assert st["pairs_true"] == int(want.sum())


def test_c2_scaled_against_oracle(env):
    torch, pa, synth, oracle = env
    A, B = synth.make_c2(seed=2, n_nuclei=600, n_vessels=40, box=160.0)
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    pairs = pa.filter_pairs(ga, gb)
    hp = pairs.cpu().numpy()
    assert np.array_equal(hp, oracle.candidate_pairs(oracle.mesh_boxes(A), oracle.mesh_boxes(B)))
    assert hp.shape[0] > 100
    want = oracle.join(A, B, hp, mode=1)
    assert 0 < want.sum() < hp.shape[0]
    for p in (0, 1):
        flags, stats, status = pa.refine(ga, gb, pairs, pa.RefineConfig(persistent=p))
        torch.cuda.synchronize()
        assert np.array_equal(flags.cpu().numpy(), want), p
    res = pa.compact(pairs, flags).cpu().numpy()
    assert np.array_equal(res, hp[want == 1])


def test_queue_overflow_decides_in_place(env):
    torch, pa, synth, oracle = env
    A, B, pairs, cls = synth.make_c4(n_pairs=60)
    want = oracle.join(A, B, pairs, mode=1)
    got, st = _run(env, A, B, pairs, persistent=1, precision=2, queue_cap=1)
    assert np.array_equal(got, want)
    assert st["queue_overflow"] > 0


def test_coordinates_outside_fp32_safe_range(env):
    """Scaling by 2^-45 is exact and keeps every answer, but puts coordinates
    below 2^-40, which disables the FP32 bounds (all tests go exact)."""
    torch, pa, synth, oracle = env
    A, B = synth.make_c1()
    pairs = np.array([(i, j) for i in range(8) for j in range(8)], np.int32)
    want = oracle.join(A, B, pairs, mode=1)
    s = np.float32(2.0 ** -45)
    As = synth.MeshSet(A.verts * s, A.faces, A.vert_off, A.face_off)
    Bs = synth.MeshSet(B.verts * s, B.faces, B.vert_off, B.face_off)
    got, st = _run(env, As, Bs, pairs, persistent=1, precision=0)
    assert np.array_equal(got, want)
    assert st["fp32_ambiguous"] > 0


def test_swap_gives_transposed_result(env):
    torch, pa, synth, oracle = env
    A, B = synth.make_c1(seed=9)
    pairs = np.array([(i, j) for i in range(8) for j in range(8)], np.int32)
    g1, _ = _run(env, A, B, pairs)
    g2, _ = _run(env, B, A, pairs[:, ::-1].copy())
    assert np.array_equal(g1, g2)


def test_deterministic_reruns(env):
    torch, pa, synth, oracle = env
    A, B, pairs, cls = synth.make_c4(n_pairs=100)
    r = [_run(env, A, B, pairs, persistent=1)[0] for _ in range(3)]
    assert all(np.array_equal(r[0], x) for x in r[1:])


def test_tiny_meshes_and_empty_pairs(env):
    torch, pa, synth, oracle = env
    tri = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64), np.array([[0, 1, 2]]))
    quad = (np.array([[0, 0, 0.5], [1, 0, 0.5], [0, 1, -0.5], [1, 1, -0.5]], np.float64), np.array([[0, 1, 2], [1, 3, 2]]))
    far = (np.array([[5, 5, 5], [6, 5, 5], [5, 6, 5]], np.float64), np.array([[0, 1, 2]]))
    A = synth.concat_meshes([tri, quad, far])
    B = synth.concat_meshes([quad, tri, far, tri])
    pairs = np.array([(i, j) for i in range(3) for j in range(4)], np.int32)
    want = oracle.join(A, B, pairs, mode=0)
    for w in (2, 4, 8):
        got, _ = _run(env, A, B, pairs, width=w, leaf=1)
        assert np.array_equal(got, want), w
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    flags, stats, status = pa.refine(ga, gb, np.zeros((0, 2), np.int32))
    torch.cuda.synchronize()
    assert flags.numel() == 0 and int(status.item()) == 0


def test_bad_pairs_and_width_mismatch_reported(env):
    torch, pa, synth, oracle = env
    A, B = synth.make_c1()
    ga, gb = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
    pairs = np.array([[0, 0], [8, 0], [0, -1], [1, 1]], np.int32)
    for p in (0, 1):
        flags, stats, status = pa.refine(ga, gb, pairs, pa.RefineConfig(persistent=p))
        torch.cuda.synchronize()
        assert int(status.item()) == -1  # PR_E_ARG
        f = flags.cpu().numpy()
        assert f[1] == 0 and f[2] == 0
        want = oracle.join(A, B, pairs[[0, 3]], mode=1)
        assert f[0] == want[0] and f[3] == want[1]
    g8 = pa.MeshBlob.build(B, width=8)
    g8.width = 4  # lie about the width: the device check must catch it
    flags, stats, status = pa.refine(ga, g8, np.array([[0, 0]], np.int32))
    torch.cuda.synchronize()
    assert int(status.item()) == -5  # PR_E_UNSUPPORTED
    assert flags.cpu().numpy()[0] == 0


def test_geometry_errors_reported(env):
    torch, pa, synth, oracle = env
    good = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float64), np.array([[0, 1, 2], [0, 1, 3]]))
    collinear = (np.array([[0, 0, 0], [1, 1, 1], [2, 2, 2]], np.float64), np.array([[0, 1, 2]]))
    badid = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64), np.array([[0, 1, 3]]))
    nan = (np.array([[0, 0, 0], [np.nan, 0, 0], [0, 1, 0]], np.float64), np.array([[0, 1, 2]]))
    for bad, face in ((collinear, 2), (badid, 2), (nan, 2)):
        S = synth.concat_meshes([good, bad])
        g = pa.MeshBlob.build(S, check_status=False)
        assert g.status() == face
    g = pa.MeshBlob.build(synth.concat_meshes([good, good]), check_status=False)
    assert g.status() == -1
