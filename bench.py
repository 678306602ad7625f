"""Benchmark of the mesh-join refinement path on one MI355X.

Workload (default): the pathology-shaped dataset - 10,000 nuclei (level-4
icospheres, 5,120 triangles, r~U[3,8], 15% low-frequency noise) against
1,000 vessels (capped tubes, 64 rings x 32 sides, 4,096 triangles, r~U[2,6])
in a 1000^3 box, FP32 coordinates, seeded synthetic data standing in for the
paper's Tissue datasets.

One step = one join query on device-resident BVHs: closed-box candidate
filter, bidirectional refinement of every candidate (one persistent launch,
FP32 filter with FP64/exact re-decision), and compaction of the result.
BVH construction is timed separately (the paper excludes acceleration
structure builds from query time, Section 4.2 "Measurement").  The per-pair
launch form of the same refinement is timed beside it.

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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "refine_persistent_c2_traffic.json")
KERNEL_SOURCES = ["paper_2609_24513_amd/csrc/refine.hip", "paper_2609_24513_amd/csrc/predicates.h",
                  "paper_2609_24513_amd/csrc/common.h"]
METRIC = "refined mesh pairs/s + segment queries/s on 1 MI355X; p50/p99 join latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def make_workload(name: str):
    from paper_2609_24513_amd import synth
    if name == "c2":
        A, B = synth.make_c2()
        desc = ("pathology-shaped: 10,000 nuclei (icosphere L4, 5,120 tris, r~U[3,8], 15% noise) x "
                "1,000 vessels (Bezier tubes 64x32, 4,096 tris, r~U[2,6]) in 1000^3, FP32")
        return A, B, None, desc
    if name == "c2-small":
        A, B = synth.make_c2(n_nuclei=1000, n_vessels=100, box=464.0)
        return A, B, None, "pathology-shaped, 1/10 scale (1,000 x 100 in 464^3)"
    if name == "c1":
        A, B = synth.make_c1()
        return A, B, None, "tiny: 8 x 8 level-2 icospheres"
    if name == "c4":
        A, B, pairs, _ = synth.make_c4()
        return A, B, pairs, "precision stress: 2,000 pairs of level-4 icospheres on a 2^-10 grid"
    if name == "c3":
        A, B, pairs = synth.make_c3()
        return A, B, pairs, ("batching: 50,000 candidate pairs from a pool of 4,096 meshes (geodesic spheres and "
                             "capped tubes) with face counts log-uniform in [500, 100,000], FP32")
    raise SystemExit("unknown workload " + name)


def cpu_baseline(A, B, pairs_np, gpu_flags, budget_s: float, seed: int = 0):
    """The exact CPU oracle on a bounded random sample of the same candidates."""
    import oracle
    oracle.build(force=False)
    try:
        threads = min(16, len(os.sched_getaffinity(0)))
    except AttributeError:
        threads = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(seed)
    P = pairs_np.shape[0]
    order = rng.permutation(P)
    n = min(P, 256)
    t = time.perf_counter()
    f = oracle.join(A, B, pairs_np[order[:n]], mode=1, threads=threads)
    dt = time.perf_counter() - t
    idx = order[:n]
    if dt < budget_s and n < P:
        n2 = int(min(P, max(n, n * budget_s / max(dt, 1e-3))))
        idx = order[:n2]
        t = time.perf_counter()
        f, ntests = oracle.join(A, B, pairs_np[idx], mode=1, threads=threads, return_tests=True)
        dt = time.perf_counter() - t
    else:
        ntests = None
    agree = bool(np.array_equal(f, gpu_flags[idx]))
    return {"value": len(idx) / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d candidate pairs (seeded random), exact SAT triangle tests with exact box "
                      "sweep-and-prune, %.1f s" % (len(idx), P, dt),
            "tri_tests_per_s": (ntests / dt) if ntests else None, "gpu_agrees_on_sample": agree}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--width", type=int, default=4)
    ap.add_argument("--leaf", type=int, default=4)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=1)
    ap.add_argument("--autotune", action="store_true", help="pick width, leaf size and schedule first")
    ap.add_argument("--compare-precision", action="store_true",
                    help="also time the FP64/exact-only precision mode, batched and per pair")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: candidate pairs shard independently across GPUs, but no "
              "multi-GPU path is implemented; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_24513_amd as pa

    torch.cuda.set_device(0)
    t = time.perf_counter()
    A, B, given_pairs, desc = make_workload(args.workload)
    log("generated %s in %.1f s: %d+%d meshes, %d+%d triangles" % (
        args.workload, time.perf_counter() - t, A.n_meshes, B.n_meshes, A.faces.shape[0], B.faces.shape[0]))

    tuned = None
    if args.autotune:
        from paper_2609_24513_amd import autotune
        pairs_for_tune = given_pairs
        if pairs_for_tune is None:
            from paper_2609_24513_amd import synth
            pairs_for_tune = synth.candidate_pairs(A.aabbs(), B.aabbs()).astype(np.int32)
        tuned = autotune.tune(A, B, pairs_for_tune, log=log)
        args.width, args.leaf, args.schedule = (tuned["best"]["width"], tuned["best"]["leaf_size"],
                                                tuned["best"]["schedule"])
        log("autotune picked W=%d L=%d schedule=%d (%.1f s, cached=%s)" % (
            args.width, args.leaf, args.schedule, tuned["tune_seconds"], tuned["cached"]))

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ga = pa.MeshBlob.build(A, width=args.width, leaf_size=args.leaf, check_status=False)
    gb = pa.MeshBlob.build(B, width=args.width, leaf_size=args.leaf, check_status=False)
    ev1.record()
    torch.cuda.synchronize()
    build_ms = ev0.elapsed_time(ev1)
    assert ga.status() == -1 and gb.status() == -1, "invalid geometry"
    log("built blobs in %.1f ms (%.2f + %.2f GB)" % (build_ms, ga.blob.numel() / 1e9, gb.blob.numel() / 1e9))

    given = None if given_pairs is None else torch.as_tensor(given_pairs).cuda()
    first = pa.filter_pairs(ga, gb) if given is None else given
    P = int(first.shape[0])
    cfg_events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
    base_cfg = dict(persistent=1, precision=args.precision, schedule=args.schedule)
    ws = pa.refine_workspace(P, args.width, pa.RefineConfig(**base_cfg))
    flags = torch.empty(P, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(len(pa.STATS_FIELDS), dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    filt_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    ref_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]

    def step(k=None):
        if k is not None:
            filt_ev[k][0].record()
        pairs = pa.filter_pairs(ga, gb, cap=P) if given is None else given
        if k is not None:
            filt_ev[k][1].record()
            ref_ev[k][0].record()
        cfg = pa.RefineConfig(**base_cfg, ev_begin=None if k is None else cfg_events[k][0],
                              ev_end=None if k is None else cfg_events[k][1])
        pa.refine(ga, gb, pairs, cfg, ws=ws, flags=flags, stats=stats, status=status)
        if k is not None:
            ref_ev[k][1].record()
        res = pa.compact(pairs, flags)
        return pairs, res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done (%d steps), %d candidate pairs" % (args.warmup, P))
    t0 = time.perf_counter()
    for k in range(args.steps):
        pairs, res = step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in cfg_events]))
    refine_ms = float(np.mean([a.elapsed_time(b) for a, b in ref_ev]))
    filter_ms = float(np.mean([a.elapsed_time(b) for a, b in filt_ev]))
    assert int(status.item()) == 0
    st = pa.stats_dict(stats)
    n_true = int(res.shape[0])
    log("timed %d steps: %.3f ms/step (kernel %.3f ms, refine %.3f ms, filter %.3f ms), %d intersecting" % (
        args.steps, ms_step, kern_ms, refine_ms, filter_ms, n_true))

    W = args.width
    # algorithmic bytes of one traversal launch: every group box read by the cull,
    # the box and the 64 segments of every traced group, one node per wave-level
    # visit (28 W bytes of boxes and child references) and one triangle per
    # wave-level leaf fetch
    alg_bytes = (24 * st["groups"] + 24 * st["groups_box_pass"] + 24 * st["segments"]
                 + 28 * W * st["node_visits"] + 36 * st["tri_fetches"])
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_source_sha") == kernel_source_sha() and tr.get("workload") == args.workload:
            traffic = tr.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_refine_persistent" if args.schedule != 2 else "k_refine_wave",
                "kernel_ms": kern_ms, "algorithmic_bytes": int(alg_bytes)}

    out_pairs = pairs.cpu().numpy()
    gflags = flags.cpu().numpy()
    ea = ga.edge_counts().cpu().numpy().astype(np.int64)
    eb = gb.edge_counts().cpu().numpy().astype(np.int64)
    nominal_segments = int((ea[out_pairs[:, 0]] + eb[out_pairs[:, 1]]).sum()) if P else 0
    def one_run(persistent, precision):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fl = torch.empty(P, dtype=torch.uint8, device="cuda")
        cfg = pa.RefineConfig(persistent=persistent, precision=precision, schedule=args.schedule,
                              ev_begin=k0, ev_end=k1)
        w_ = pa.refine_workspace(P, W, cfg)
        pa.refine(ga, gb, pairs, cfg, ws=w_, flags=fl)  # warm
        torch.cuda.synchronize()
        e0.record()
        _, pst, pstatus = pa.refine(ga, gb, pairs, cfg, ws=w_, flags=fl)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        return {"refine_ms": ms, "kernels_ms": k0.elapsed_time(k1), "pairs_per_s": P / (ms * 1e-3),
                "same_flags": bool(np.array_equal(fl.cpu().numpy(), gflags)),
                "stats": pa.stats_dict(pst)}

    plain = None
    if not args.skip_plain:
        plain = one_run(0, args.precision)
        plain["launches"] = P
        plain["batched_speedup"] = plain["refine_ms"] / refine_ms
        log("plain per-pair launches: %.2f ms (%.1fx slower), same flags: %s" % (
            plain["refine_ms"], plain["batched_speedup"], plain["same_flags"]))
    precision_cmp = None
    if args.compare_precision:
        precision_cmp = {"batched_fp64_exact": one_run(1, 1)}
        if not args.skip_plain:
            precision_cmp["per_pair_fp64_exact"] = one_run(0, 1)
        for k, v in precision_cmp.items():
            log("%s: %.2f ms, same flags: %s" % (k, v["refine_ms"], v["same_flags"]))

    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(A, B, out_pairs, gflags, args.cpu_seconds)
        log("cpu oracle: %.1f pairs/s on %d threads, agrees: %s" % (cpu["value"], cpu["cores"],
                                                                     cpu["gpu_agrees_on_sample"]))

    value = P / (ms_step * 1e-3)
    line = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": desc, "workload_id": args.workload, "candidate_pairs": P,
                   "intersecting_pairs": n_true, "bvh_width": W, "leaf_size": args.leaf,
                   "precision": ["fp32 filter + fp64/exact fallback", "fp64/exact", "forced deferral"][args.precision],
                   "refine": "one persistent launch (batched)", "schedule": args.schedule,
                   "step": ("filter + refine + compact" if given is None else "refine + compact (pairs given)")},
        "segment_queries_per_s": st["segments"] / (refine_ms * 1e-3),
        "nominal_segments": nominal_segments,
        "nominal_segment_queries_per_s": nominal_segments / (refine_ms * 1e-3),
        "refine_pairs_per_s": P / (refine_ms * 1e-3),
        "refine_ms": refine_ms, "filter_ms": filter_ms, "build_ms": build_ms,
        "roofline": roofline, "cpu_baseline": cpu, "plain_per_pair": plain,
        "precision_comparison": precision_cmp, "autotune": tuned,
        "stats": st,
        "retest_fraction": (st["fp32_ambiguous"] / st["tri_tests"]) if st["tri_tests"] else 0.0,
    }
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.calibrate_copy_mib)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
