"""Benchmark of the mesh-join refinement path on one MI355X.

Headline workload (default): the batching workload - 50,000 candidate pairs
drawn from a pool of 4,096 meshes (noise-displaced geodesic spheres and
capped tubes) whose face counts are log-uniform in [500, 100,000], all
refined in one persistent launch, FP32 filter with FP64/exact re-decision.
It is the largest configuration that fits one GPU.  The BVH width, leaf size
and schedule come from the autotuner (2% stratified sample).

One step = one pass of the hot path over the batch, inputs resident in HBM:
bidirectional refinement of every given candidate pair and compaction of
the result (for workloads without a given pair list the closed-box filter
runs first).  BVH construction is timed separately (the paper excludes
acceleration-structure builds from query time, Section 4.2 "Measurement").

Reported beside the headline: segment queries/s, the roofline object of the
traversal kernels, the per-pair launch form of the same refinement, the
FP64/exact-only precision mode batched and per pair, the exact CPU oracle on
a bounded sample, and, under "workloads", the pathology-shaped workload
(filter + refine + compaction), the precision-stress workload (re-test
fraction, mismatches against the oracle) and the serving workload (p50/p99
latency at 50, 200 and 1,000 requests/s against first-in first-out per-pair
launches on the same trace).

Prints ONE JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "refine_traversal_%s_traffic.json")  # % workload
KERNEL_SOURCES = ["paper_2609_24513_amd/csrc/refine.hip", "paper_2609_24513_amd/csrc/predicates.h",
                  "paper_2609_24513_amd/csrc/common.h", "paper_2609_24513_amd/csrc/build.hip"]
METRIC = "refined mesh pairs/s + segment queries/s on 1 MI355X; p50/p99 join latency"
SCHEDULE_NAMES = {0: "auto", 1: "wave-per-pair", 2: "wave-per-segment"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace runs collapsed, so that
    an edit of a comment does not count as a change of the kernels."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            i = text.find("\n", i)
            i = n if i < 0 else i
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c == '"' or c == "'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(_code_only(open(os.path.join(ROOT, f), encoding="utf-8").read()).encode())
    return h.hexdigest()


DESCS = {
    "c2": ("pathology-shaped: 10,000 nuclei (icosphere L4, 5,120 tris, r~U[3,8], 15% noise) x 1,000 vessels "
           "(Bezier tubes 64x32, 4,096 tris, r~U[2,6]) in 1000^3, FP32"),
    "c2-small": "pathology-shaped, 1/10 scale (1,000 x 100 in 464^3)",
    "c1": "tiny: 8 x 8 level-2 icospheres",
    "c3": ("batching: 50,000 candidate pairs from a pool of 4,096 meshes (geodesic spheres and capped tubes) with "
           "face counts log-uniform in [500, 100,000], FP32"),
    "c4": "precision stress: 2,000 pairs of level-4 icospheres on a 2^-10 grid (30% tangent, 20% coplanar, "
          "10% vertex on surface, 40% random)",
}
for _k, _m in enumerate((4, 20, 39, 74, 144)):
    DESCS["sweep%d" % _k] = ("mesh complexity: 500 x 500 unit UV spheres (%d rings x %d segments, %d triangles each) "
                             "at fixed placements, 100 intersecting pairs" % (_m, 2 * _m, 2 * ((_m - 1) * 2 * _m + 2) - 4))


def make_workload(name: str):
    from paper_2609_24513_amd import synth
    if name == "c2":
        A, B = synth.make_c2()
        return A, B, None
    if name == "c2-small":
        A, B = synth.make_c2(n_nuclei=1000, n_vessels=100, box=464.0)
        return A, B, None
    if name == "c1":
        A, B = synth.make_c1()
        return A, B, None
    if name == "c4":
        A, B, pairs, _ = synth.make_c4()
        return A, B, pairs
    if name == "c3":
        return synth.make_c3()
    if name.startswith("sweep") and name[5:].isdigit() and int(name[5:]) < len(synth.SWEEP_RINGS):
        A, B = synth.make_sweep(int(name[5:]))
        return A, B, None
    raise SystemExit("unknown workload " + name)


def achievable_hbm_gbs(torch, mib: int = 2048, reps: int = 5) -> float:
    """Streaming device-to-device copy of `mib` MiB on the same GPU: bytes read plus
    bytes written over the best of `reps` timed copies."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / best / 1e9


def cpu_baseline(A, B, pairs_np, gpu_flags, budget_s: float, seed: int = 0):
    """The exact CPU oracle, as it stands, on a bounded random sample of the
    same candidates (about budget_s seconds of work), with the oracle's default
    thread count: the host cores this process may use, at most 16 (the CPU
    share of one GPU on the GPU hosts)."""
    import oracle
    oracle.build(force=False)
    threads = oracle.default_threads()
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    rng = np.random.default_rng(seed)
    P = pairs_np.shape[0]
    order = rng.permutation(P)
    n = min(P, 128)
    t = time.perf_counter()
    f = oracle.join(A, B, pairs_np[order[:n]], mode=1, threads=threads)
    dt = time.perf_counter() - t
    idx = order[:n]
    ntests = None
    if dt < budget_s / 4 and n < P:
        n2 = int(min(P, max(n, n * budget_s / max(dt, 1e-3))))
        idx = order[:n2]
        t = time.perf_counter()
        f, ntests = oracle.join(A, B, pairs_np[idx], mode=1, threads=threads, return_tests=True)
        dt = time.perf_counter() - t
    if dt < budget_s / 2 and len(idx) < P:  # the first estimate came out short: scale once more
        n3 = int(min(P, len(idx) * budget_s / max(dt, 1e-3)))
        idx = order[:n3]
        t = time.perf_counter()
        f, ntests = oracle.join(A, B, pairs_np[idx], mode=1, threads=threads, return_tests=True)
        dt = time.perf_counter() - t
    agree = bool(np.array_equal(f, gpu_flags[idx]))
    # single-thread rate on a sub-sample of about a quarter of the budget
    n1 = int(min(len(idx), max(16, len(idx) * (0.25 * budget_s) / max(dt * threads, 1e-3))))
    t = time.perf_counter()
    f1 = oracle.join(A, B, pairs_np[idx[:n1]], mode=1, threads=1)
    dt1 = time.perf_counter() - t
    agree = agree and bool(np.array_equal(f1, gpu_flags[idx[:n1]]))
    return {"value": len(idx) / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "host_cores_visible": visible,
            "single_thread_pairs_per_s": n1 / dt1, "single_thread_sample": n1,
            "sample": "%d of %d candidate pairs (seeded random), exact SAT triangle tests with exact box "
                      "sweep-and-prune, %d threads, %.1f s" % (len(idx), P, threads, dt),
            "tri_tests_per_s": (ntests / dt) if ntests else None, "gpu_agrees_on_sample": agree}


def roofline_of(st: dict, W: int, kern_ms: float, workload: str, L: int = 0, sched: int = 1) -> dict:
    """Roofline of the traversal kernels of one refinement pass.  Algorithmic
    bytes: 24 B per segment started, 28 W B per (wave-level) node visit, 36 B
    per segment-triangle test.  Also the bytes the kernels' loads cover as
    issued (group boxes in the cull, segments of traced groups, nodes, leaf
    triangles once per wave)."""
    alg = 24 * st["segments"] + 28 * W * st["node_visits"] + 36 * st["tri_tests"]
    loaded = (24 * st["groups"] + 24 * st["groups_box_pass"] + 24 * st["segments"]
              + 28 * W * st["node_visits"] + 36 * st["tri_fetches"])
    achieved = alg / (kern_ms * 1e-3) / 1e9
    traffic = None
    valu = None
    path = TRAFFIC_FILE % workload
    if os.path.exists(path):
        doc = json.load(open(path))
        sha = kernel_source_sha()
        for tr in doc.get("entries", [doc]):
            if (tr.get("kernel_source_sha") == sha and tr.get("workload") == workload
                    and (tr.get("bvh_width"), tr.get("leaf_size"), tr.get("schedule")) == (W, L, sched)):
                traffic = tr.get("hbm_bytes_per_launch")
                valu = tr.get("valu_use")
    # valu_use: share of SIMD cycles issuing vector instructions, per kernel,
    # from the profiled run's counters (4 x SQ_INSTS_VALU / SIMD cycles)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_cull + k_trace",
            "kernel_ms": kern_ms, "algorithmic_bytes": int(alg), "loaded_bytes_model": int(loaded),
            "loaded_gbs": loaded / (kern_ms * 1e-3) / 1e9, "valu_use": valu}


def predicate_bench(torch, pa, ga, gb, pairs, cfg_kw: dict, reps: int = 5) -> dict:
    """The four join predicates on the same candidate pairs (Sections 3.2-3.4),
    each one refine_predicate call (edge tracing, then for contains / within /
    intersection the point-in-mesh rays on the pairs without a shared point):
    the mean time of `reps` calls after one warm-up, the containment phase as
    the difference to the overlap predicate, the result counts and the ray
    statistics; and each predicate's flags against the two phases run as
    separate calls (refine, then inside_pairs in the predicate's mode)."""
    P = int(pairs.shape[0])
    cfg = pa.RefineConfig(**cfg_kw)
    ws = pa.predicate_workspace(P, ga.width, cfg)
    flags = torch.empty(P, dtype=torch.uint8, device="cuda")
    st = torch.zeros(len(pa.STATS_FIELDS), dtype=torch.int64, device="cuda")
    ist = torch.zeros(len(pa.INSIDE_FIELDS), dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e in [e for pair in evs for e in pair]:
        e.record()
    res = {}
    for name, code in pa.PREDICATES.items():
        for r in range(-1, reps):
            if r >= 0:
                evs[r][0].record()
            pa.predicate(ga, gb, pairs, code, cfg, ws=ws, flags=flags, stats=st, istats=ist, status=status)
            if r >= 0:
                evs[r][1].record()
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        got = flags.cpu().numpy()[:P].copy()
        total = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        cross, _, _ = pa.refine(ga, gb, pairs, cfg)
        sep = pa.inside(ga, gb, pairs, mode=code, cross=cross)[0] if code else cross
        torch.cuda.synchronize()
        r_ = {"ms": total, "result_pairs": int(got.sum()), "pairs_per_s": P / (total * 1e-3),
              "same_as_separate_calls": bool(np.array_equal(sep.cpu().numpy()[:P], got))}
        if code:
            r_["containment_rays_ms"] = total - res["overlap"]["ms"]
            r_["inside_stats"] = pa.inside_stats_dict(ist)
        res[name] = r_
        log("predicate %-12s %.3f ms (containment rays %.3f), %d pairs" % (
            name, total, r_.get("containment_rays_ms", 0.0), r_["result_pairs"]))
    del ws
    return res


def run_join(name: str, args, tune: bool, plain: bool, compare_precision: bool, cpu: bool, steps: int,
             warmup: int, check_oracle: bool = False, predicates: bool = False) -> dict:
    """Times one join workload: returns the measurements as a dict."""
    import torch
    import paper_2609_24513_amd as pa
    t = time.perf_counter()
    A, B, given_pairs = make_workload(name)
    gen_s = time.perf_counter() - t
    log("%s: generated in %.1f s: %d+%d meshes, %d+%d triangles" % (
        name, gen_s, A.n_meshes, B.n_meshes, A.faces.shape[0], B.faces.shape[0]))
    W, L, sched, table = args.width, args.leaf, args.schedule, 0
    tuned = None
    if tune:
        from paper_2609_24513_amd import autotune
        pairs_for_tune = given_pairs
        if pairs_for_tune is None:
            g4a, g4b = pa.MeshBlob.build(A), pa.MeshBlob.build(B)
            pairs_for_tune = pa.filter_pairs(g4a, g4b).cpu().numpy()
            del g4a, g4b
        tuned = autotune.tune(A, B, pairs_for_tune, frac=args.tune_frac, log=log,
                              prefer=(args.width, args.leaf, args.schedule))
        W, L, sched = tuned["best"]["width"], tuned["best"]["leaf_size"], tuned["best"]["schedule"]
        table = tuned["best"].get("seg_live_max", 0)
        log("%s: autotune picked W=%d L=%d schedule=%d table=%08x (%.1f s, cached=%s)" % (
            name, W, L, sched, table, tuned["tune_seconds"], tuned["cached"]))
        tuned = {k: tuned[k] for k in ("best", "per_bucket", "sample", "tune_seconds", "cached")}

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the meshes are resident in HBM before the build is timed, and one
    # untimed build first leaves its device memory in the allocator's cache
    # (the library allocates nothing itself)
    import types
    da, db = (types.SimpleNamespace(**{k: torch.as_tensor(getattr(S, k)).cuda()
                                       for k in ("verts", "faces", "vert_off", "face_off")}) for S in (A, B))
    ga = pa.MeshBlob.build(da, width=W, leaf_size=L, check_status=False)
    gb = pa.MeshBlob.build(db, width=W, leaf_size=L, check_status=False)
    torch.cuda.synchronize()
    del ga, gb
    ev0.record()
    ga = pa.MeshBlob.build(da, width=W, leaf_size=L, check_status=False)
    gb = pa.MeshBlob.build(db, width=W, leaf_size=L, check_status=False)
    ev1.record()
    torch.cuda.synchronize()
    build_ms = ev0.elapsed_time(ev1)
    assert ga.status() == -1 and gb.status() == -1, "invalid geometry"
    log("%s: built blobs in %.1f ms (%.2f + %.2f GB)" % (name, build_ms, ga.blob.numel() / 1e9,
                                                         gb.blob.numel() / 1e9))

    given = None if given_pairs is None else torch.as_tensor(given_pairs).cuda()
    first = pa.filter_pairs(ga, gb) if given is None else given
    P = int(first.shape[0])
    kern_events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(steps)]
    base_cfg = dict(persistent=1, precision=args.precision, schedule=sched, seg_live_max=table,
                    trace_budget=args.trace_budget)
    ws = pa.refine_workspace(P, W, pa.RefineConfig(**base_cfg))
    flags = torch.empty(P, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(len(pa.STATS_FIELDS), dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    n_split = min(steps, 5)
    filt_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_split)]
    ref_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_split)]

    def step(k=None, split=None):
        # one pass on the device: (filter ->) refine -> compaction, the pair count
        # handed from stage to stage on the device (no host round trip).  The
        # kernel events ride on the dispatches themselves; the stage-split
        # events (`split`) insert marker packets and are only used outside the
        # timed loop.
        if split is not None:
            filt_ev[split][0].record()
        if given is None:
            pairs, cnt = pa.filter_pairs(ga, gb, cap=P, sync=False)
        else:
            pairs, cnt = given, None
        if split is not None:
            filt_ev[split][1].record()
            ref_ev[split][0].record()
        cfg = pa.RefineConfig(**base_cfg, ev_begin=None if k is None else kern_events[k][0],
                              ev_end=None if k is None else kern_events[k][1], n_dev=cnt)
        pa.refine(ga, gb, pairs, cfg, ws=ws, flags=flags, stats=stats, status=status)
        if split is not None:
            ref_ev[split][1].record()
        res, rcnt = pa.compact(pairs, flags, n_dev=cnt, sync=False)
        return pairs, cnt, res, rcnt

    # torch creates an event at its first record: create them all here, so
    # that no marker packet lands inside the timed loop
    for e in [e for pair in kern_events + filt_ev + ref_ev for e in pair]:
        e.record()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        pairs, cnt, res, rcnt = step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if cnt is not None and int(cnt.item()) != P:
        raise RuntimeError("filter count %d != %d" % (int(cnt.item()), P))
    res = res[:int(rcnt.item())]
    ms_step = (t1 - t0) * 1e3 / steps
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in kern_events]))
    for k in range(len(filt_ev)):
        step(split=k)
    torch.cuda.synchronize()
    refine_ms = float(np.mean([a.elapsed_time(b) for a, b in ref_ev]))
    filter_ms = float(np.mean([a.elapsed_time(b) for a, b in filt_ev])) if given is None else 0.0
    assert int(status.item()) == 0
    st = pa.stats_dict(stats)
    n_true = int(res.shape[0])
    log("%s: %d steps: %.3f ms/step (traversal kernels %.3f ms, refine %.3f ms, filter %.3f ms), %d of %d "
        "intersecting" % (name, steps, ms_step, kern_ms, refine_ms, filter_ms, n_true, P))

    roof = roofline_of(st, W, kern_ms, name, L, sched)
    out_pairs = pairs.cpu().numpy()[:P]
    gflags = flags.cpu().numpy()[:P]
    ea = ga.edge_counts().cpu().numpy().astype(np.int64)
    eb = gb.edge_counts().cpu().numpy().astype(np.int64)
    nominal_segments = int((ea[out_pairs[:, 0]] + eb[out_pairs[:, 1]]).sum()) if P else 0

    def one_run(persistent, precision):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fl = torch.empty(P, dtype=torch.uint8, device="cuda")
        cfg = pa.RefineConfig(persistent=persistent, precision=precision, schedule=sched, seg_live_max=table,
                              ev_begin=k0, ev_end=k1)
        w_ = pa.refine_workspace(P, W, cfg)
        pa.refine(ga, gb, first, cfg, ws=w_, flags=fl)  # warm
        torch.cuda.synchronize()
        e0.record()
        _, pst, pstatus = pa.refine(ga, gb, first, cfg, ws=w_, flags=fl)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        assert int(pstatus.item()) == 0
        return {"refine_ms": ms, "kernels_ms": k0.elapsed_time(k1), "pairs_per_s": P / (ms * 1e-3),
                "same_flags": bool(np.array_equal(fl.cpu().numpy()[:P], gflags)), "stats": pa.stats_dict(pst)}

    plain_r = None
    if plain:
        plain_r = one_run(0, args.precision)
        plain_r["launches"] = P
        plain_r["batched_speedup"] = plain_r["refine_ms"] / refine_ms
        log("%s: per-pair launches %.2f ms (batched is %.1fx faster), same flags: %s" % (
            name, plain_r["refine_ms"], plain_r["batched_speedup"], plain_r["same_flags"]))
    prec = None
    if compare_precision:
        prec = {"batched_fp32_fp64_fallback_ms": refine_ms, "batched_fp64_exact": one_run(1, 1)}
        if plain:
            prec["per_pair_fp32_fp64_fallback_ms"] = plain_r["refine_ms"]
            prec["per_pair_fp64_exact"] = one_run(0, 1)
            prec["speedup_batched_fp32_over_per_pair_fp64"] = prec["per_pair_fp64_exact"]["refine_ms"] / refine_ms
        prec["speedup_fp32_fallback_over_fp64_exact_batched"] = prec["batched_fp64_exact"]["refine_ms"] / refine_ms
        for k, v in prec.items():
            if isinstance(v, dict):
                log("%s: %s %.2f ms, same flags: %s" % (name, k, v["refine_ms"], v["same_flags"]))
    cpu_r = None
    if cpu:
        cpu_r = cpu_baseline(A, B, out_pairs, gflags, args.cpu_seconds)
        log("%s: cpu oracle %.1f pairs/s on %d threads, agrees: %s" % (
            name, cpu_r["value"], cpu_r["cores"], cpu_r["gpu_agrees_on_sample"]))
    preds = None
    if predicates:
        preds = predicate_bench(torch, pa, ga, gb, first, base_cfg)
    oracle_check = None
    if check_oracle:
        import oracle
        t = time.perf_counter()
        want = oracle.join(A, B, out_pairs, mode=1)
        oracle_check = {"pairs": P, "mismatches": int((want != gflags).sum()),
                        "oracle_true": int(want.sum()), "oracle_s": time.perf_counter() - t}
        log("%s: oracle on every pair: %d mismatches" % (name, oracle_check["mismatches"]))
    out = {
        "workload": DESCS[name], "workload_id": name, "candidate_pairs": P, "intersecting_pairs": n_true,
        "bvh_width": W, "leaf_size": L, "schedule": sched, "schedule_name": SCHEDULE_NAMES.get(sched, str(sched)),
        "seg_live_max": table,
        "precision": ["fp32 filter + fp64/exact fallback", "fp64/exact", "forced deferral"][args.precision],
        "step": ("filter + refine + compact" if given is None else "refine + compact (pairs given)"),
        "ms_per_step": ms_step, "pairs_per_s": P / (ms_step * 1e-3),
        "refine_ms": refine_ms, "filter_ms": filter_ms, "traversal_kernels_ms": kern_ms,
        "refine_pairs_per_s": P / (refine_ms * 1e-3),
        "segment_queries_per_s": st["segments"] / (refine_ms * 1e-3),
        "nominal_segments": nominal_segments,
        "nominal_segment_rate_per_s": nominal_segments / (refine_ms * 1e-3),
        "build_ms": build_ms, "generate_s": gen_s, "roofline": roof, "plain_per_pair": plain_r,
        "precision_comparison": prec, "autotune": tuned, "cpu_baseline": cpu_r, "stats": st,
        "retest_fraction": (st["fp32_ambiguous"] / st["tri_tests"]) if st["tri_tests"] else 0.0,
        "oracle_check": oracle_check, "predicates": preds,
        "triangles_per_mesh": int(A.faces.shape[0] // max(A.n_meshes, 1)),
    }
    del ga, gb, ws, given, first, da, db
    torch.cuda.empty_cache()
    return out


def serve_bench(args) -> dict:
    """Serving: 50,000 resident level-2 icospheres (two datasets of 25,000, split
    by id parity), Poisson arrivals at several rates, each request a query box
    selecting 1-5,000 candidate pairs.  Continuous batching (persistent refine
    per batch) against first-in first-out per-pair launches on the same trace."""
    import torch
    import paper_2609_24513_amd as pa
    from paper_2609_24513_amd import serve, synth
    t = time.perf_counter()
    R, S = synth.make_c5_pool()
    gr = pa.MeshBlob.build(R, width=4, leaf_size=4)
    gs = pa.MeshBlob.build(S, width=4, leaf_size=4)
    br, bs = R.aabbs(), S.aabbs()
    log("serving pool ready in %.1f s: %d + %d meshes" % (time.perf_counter() - t, R.n_meshes, S.n_meshes))
    n = args.serve_requests
    rates = [(50.0, max(8, n // 4)), (200.0, max(8, n // 2)), (1000.0, n)]
    out = {}
    for lam, nreq in rates:
        trace = serve.make_trace(br, bs, nreq, lam, seed=5)
        srv = serve.JoinServer(gr, gs, max_req_per_batch=32, slots=3, hbm_budget=args.hbm_budget)
        srv.run([serve.Request(r.rid, r.t_arrival, r.box) for r in trace[:8]], realtime=False)  # warm-up
        srv.batches = 0
        srv.max_in_flight = 0
        served = srv.run(trace)
        s1 = serve.latency_summary(served)
        s1["batches"] = srv.batches
        s1["max_slots_in_flight"] = srv.max_in_flight
        s1["slots"] = len(srv.slots)
        s1["slot_bytes"] = srv.slot_bytes
        plain_trace = [serve.Request(r.rid, r.t_arrival, r.box) for r in trace[:args.plain_requests]]
        plain = serve.run_plain(gr, gs, plain_trace)
        s2 = serve.latency_summary(plain)
        same = all(np.array_equal(a.flags, b.flags) and np.array_equal(a.pairs, b.pairs)
                   for a, b in zip(served[:len(plain)], plain))
        out["%g" % lam] = {"served": s1, "plain_fifo_per_pair": s2, "same_results": bool(same)}
        log("serving lambda=%g/s: p50 %.2f ms p99 %.2f ms %.0f pairs/s (%d batches); plain FIFO p50 %.2f p99 %.2f ms;"
            " same %s" % (lam, s1["p50_ms"], s1["p99_ms"], s1["pairs_per_s"], srv.batches, s2["p50_ms"],
                          s2["p99_ms"], same))
    # saturation: the whole highest-rate trace released at once (closed loop)
    trace = serve.make_trace(br, bs, n, 1000.0, seed=6)
    srv = serve.JoinServer(gr, gs, max_req_per_batch=32, slots=3, hbm_budget=args.hbm_budget)
    sat = serve.latency_summary(srv.run(trace, realtime=False))
    sat["batches"] = srv.batches
    out["saturation"] = sat
    log("serving saturation: %.0f pairs/s, %.0f requests/s over %d batches" % (
        sat["pairs_per_s"], sat["requests"] / sat["span_s"], srv.batches))
    del gr, gs
    torch.cuda.empty_cache()
    top = out["1000"]["served"]
    return {"workload": "serving: 2 x 25,000 resident level-2 icospheres in 58.5^3, Poisson arrivals, query boxes "
                        "selecting 1-5,000 candidate pairs, batches of up to 32 requests on 3 streams",
            "p50_ms": {k: v["served"]["p50_ms"] for k, v in out.items() if k != "saturation"},
            "p99_ms": {k: v["served"]["p99_ms"] for k, v in out.items() if k != "saturation"},
            "plain_fifo_p50_ms": {k: v["plain_fifo_per_pair"]["p50_ms"] for k, v in out.items() if k != "saturation"},
            "plain_fifo_p99_ms": {k: v["plain_fifo_per_pair"]["p99_ms"] for k, v in out.items()
                                  if k != "saturation"},
            "pairs_per_s_at_1000": top["pairs_per_s"], "saturation_pairs_per_s": sat["pairs_per_s"],
            "same_results_as_plain": all(v["same_results"] for k, v in out.items() if k != "saturation"),
            "detail": out}


def _time_pairs_path(torch, pa, ga, gb, reps=3):
    """Per-pair path (filter -> refine -> compact) time and result count."""
    def run():
        pairs = pa.filter_pairs(ga, gb)
        # a survivor queue large enough for one group per unit of 2^25 pairs
        flags, _, _ = pa.refine(ga, gb, pairs, pa.RefineConfig(schedule=1, survivor_cap=1 << 26))
        return pa.compact(pairs, flags)
    run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        res = run()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), res.cpu().numpy()


def dataset_bench(args) -> dict:
    """The paper's dataset-level design against the per-pair path, and its
    materialisation strategies (Sections 3.2, 3.5; Fig. 5): 50,000 x 50,000
    axis-aligned cubes at three universe sizes (join selectivity about
    1e-4, 1e-3, 1e-2), and the pathology-shaped workload."""
    import torch
    import paper_2609_24513_amd as pa
    from paper_2609_24513_amd import dataset as ds, synth
    out = {"workload": "50,000 x 50,000 axis-aligned cubes (sides U[1, 2]) in a universe whose side sets the "
                       "selectivity; then the pathology-shaped workload", "rows": []}
    W, L = 4, 4
    plans = [("cubes", side) for side in (63.0, 28.5, 12.4)] + [("c2", None)]
    for name, side in plans:
        t = time.perf_counter()
        if name == "cubes":
            A, B = synth.make_cubes(50_000, side)
        else:
            A, B, _ = make_workload("c2")
        ga, gb = pa.MeshBlob.build(A, width=W, leaf_size=L), pa.MeshBlob.build(B, width=W, leaf_size=L)
        tb0 = time.perf_counter()
        da, db = ds.DatasetBlob.build(A, width=8, leaf_size=2), ds.DatasetBlob.build(B, width=8, leaf_size=2)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - tb0
        ma, mb = ds.max_groups(A), ds.max_groups(B)
        pp_ms, ref = _time_pairs_path(torch, pa, ga, gb)
        row = {"workload": name, "universe_side": side, "objects": [A.n_meshes, B.n_meshes],
               "triangles": [int(A.faces.shape[0]), int(B.faces.shape[0])], "result_pairs": int(ref.shape[0]),
               "selectivity": ref.shape[0] / (A.n_meshes * B.n_meshes), "per_pair_path_ms": pp_ms,
               "dataset_blob_build_s": build_s, "strategies": {}}
        for strat in ("estimated", "two_pass", "fixed"):
            kw = {"fixed_slots": 1 << 28} if strat == "fixed" else {}
            ds.join_dataset(ga, gb, da, db, ma, mb, strategy=strat, **kw)  # warm-up
            runs = [ds.join_dataset(ga, gb, da, db, ma, mb, strategy=strat, **kw) for _ in range(3)]
            got, info = runs[-1]
            ms = float(np.median([r[1]["ms"] for r in runs]))
            info = {k: v for k, v in info.items() if k not in ("stats_ab", "stats_ba")}
            info.update({"ms": ms, "same_pairs_as_per_pair_path": bool(np.array_equal(got, ref)),
                         "records": info.get("records", runs[-1][1]["stats_ab"]["records"] +
                                             runs[-1][1]["stats_ba"]["records"])})
            row["strategies"][strat] = info
            log("dataset-level %s %s: %s %.2f ms (per-pair path %.2f ms), %d pairs, output %.1f MB, same: %s" % (
                name, "" if side is None else "side %.1f" % side, strat, ms, pp_ms, info["pairs"],
                info["output_bytes"] / 1e6, info["same_pairs_as_per_pair_path"]))
        out["rows"].append(row)
        log("dataset-level %s: generated + built in %.1f s" % (name, time.perf_counter() - t))
        del ga, gb, da, db
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", help="headline workload: c3 (default), c2, c4, c2-small, c1, c5")
    ap.add_argument("--width", type=int, default=8, help="BVH width (the autotuner keeps it unless another "
                                                           "configuration is more than 3%% faster)")
    ap.add_argument("--leaf", type=int, default=1)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=1, help="0 auto, 1 wave-per-pair, 2 wave-per-segment")
    ap.add_argument("--trace-budget", type=int, default=0,
                    help="0 = library default (waves of a block share pending subtrees), > 0 = steps before a long "
                         "group hands its stack to a continuation pass, -1 = no hand-over")
    ap.add_argument("--no-tune", action="store_true", help="use --width/--leaf/--schedule instead of the autotuner")
    ap.add_argument("--tune-frac", type=float, default=1.0,
                    help="autotuner sample (stratified by pair size; smaller samples were launch-latency bound "
                         "and ranked widths differently from the whole batch); the blob builds dominate its time")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests at the highest serving rate")
    ap.add_argument("--plain-requests", type=int, default=200, help="requests replayed on the plain path")
    ap.add_argument("--hbm-budget", type=int, default=1 << 30, help="serving: HBM bytes for in-flight requests")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-dataset", action="store_true", help="skip the dataset-level design study")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (candidate pairs shard independently "
              "across GPUs, but nothing here launches more than one); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.workload == "c5":
        r = serve_bench(args)
        line = {"metric": METRIC, "value": r["pairs_per_s_at_1000"], "unit": "pairs/s", "n_gpus": 1,
                "steps": args.serve_requests, "warmup": 8, "ms_per_step": None, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
                "config": {"workload": r["workload"], "workload_id": "c5"}, "serving": r}
        print(json.dumps(line), flush=True)
        return

    head = run_join(args.workload, args, tune=not args.no_tune, plain=not args.skip_plain,
                    compare_precision=not args.skip_plain, cpu=not args.skip_cpu, steps=args.steps,
                    warmup=args.warmup, predicates=True)
    head["roofline"]["achievable_gbs"] = achievable_hbm_gbs(torch)
    head["roofline"]["frac_of_achievable"] = head["roofline"]["achieved"] / head["roofline"]["achievable_gbs"]
    extras = {}
    # the other workloads run untuned at width 4 / leaf 4
    xargs = argparse.Namespace(**vars(args))
    xargs.width, xargs.leaf, xargs.schedule = 4, 4, 1
    if not args.no_extras:
        if args.workload != "c2":
            extras["c2"] = run_join("c2", xargs, tune=False, plain=False, compare_precision=False, cpu=False,
                                    steps=args.steps, warmup=args.warmup, predicates=True)
        if args.workload != "c4":
            extras["c4"] = run_join("c4", xargs, tune=False, plain=not args.skip_plain,
                                    compare_precision=not args.skip_plain, cpu=False, steps=args.steps,
                                    warmup=args.warmup, check_oracle=True)
        extras["c5"] = serve_bench(args)
        sweep = []
        for k in range(5):
            r = run_join("sweep%d" % k, xargs, tune=False, plain=False, compare_precision=False, cpu=False,
                         steps=args.steps, warmup=args.warmup)
            sweep.append({"triangles_per_sphere": r["triangles_per_mesh"], "ms_per_step": r["ms_per_step"],
                          "refine_ms": r["refine_ms"], "filter_ms": r["filter_ms"],
                          "candidate_pairs": r["candidate_pairs"], "intersecting_pairs": r["intersecting_pairs"],
                          "segment_queries_per_s": r["segment_queries_per_s"], "build_ms": r["build_ms"]})
        extras["mesh_complexity"] = {"workload": "500 x 500 unit UV spheres at fixed placements, tessellation "
                                                 "swept over five stages (Section 4.4)", "stages": sweep}
        if not args.skip_dataset:
            extras["dataset_level"] = dataset_bench(args)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.calibrate_copy_mib)

    def brief(r):
        keys = ("workload", "candidate_pairs", "intersecting_pairs", "bvh_width", "leaf_size", "schedule_name",
                "step", "ms_per_step", "pairs_per_s", "refine_ms", "filter_ms", "refine_pairs_per_s",
                "segment_queries_per_s", "traversal_kernels_ms", "build_ms", "retest_fraction", "roofline",
                "oracle_check", "plain_per_pair", "precision_comparison", "stats", "predicates")
        return {k: r[k] for k in keys if k in r}

    line = {
        "metric": METRIC, "value": head["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": head["workload"], "workload_id": head["workload_id"],
                   "candidate_pairs": head["candidate_pairs"], "intersecting_pairs": head["intersecting_pairs"],
                   "bvh_width": head["bvh_width"], "leaf_size": head["leaf_size"],
                   "schedule": head["schedule_name"], "precision": head["precision"],
                   "refine": "one persistent launch (batched)", "step": head["step"]},
        "segment_queries_per_s": head["segment_queries_per_s"],
        "refine_pairs_per_s": head["refine_pairs_per_s"], "refine_ms": head["refine_ms"],
        "nominal_segments": head["nominal_segments"], "nominal_segment_rate_per_s": head["nominal_segment_rate_per_s"],
        "build_ms": head["build_ms"],
        "roofline": head["roofline"], "cpu_baseline": head["cpu_baseline"],
        "plain_per_pair": head["plain_per_pair"], "precision_comparison": head["precision_comparison"],
        "autotune": head["autotune"], "stats": head["stats"], "retest_fraction": head["retest_fraction"],
        "predicates": head["predicates"],
        "workloads": {k: (brief(v) if k not in ("c5", "mesh_complexity", "dataset_level") else v)
                      for k, v in extras.items()},
    }
    if "c5" in extras:
        line["p50_ms"] = extras["c5"]["p50_ms"]
        line["p99_ms"] = extras["c5"]["p99_ms"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
