"""Autotuner for the batched refinement: BVH width, leaf size and schedule.

For a workload (two mesh datasets and their candidate pairs) it draws a
seeded sample stratified by pair size (F_A + F_B, log-spaced buckets), builds
the blobs once per (width, leaf size), times the persistent refinement of the
sample for every schedule with HIP events - wave-per-pair, wave-per-segment,
and the automatic schedule with per-target-size tables that send groups with
few segments near the target wave-per-segment - and returns the
configuration with the lowest time over the whole sample, plus the winners
per pair-size bucket.  Results are cached in a JSON file keyed by device
name, library build (hash of libpierce_hip.so) and workload digest.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, Optional, Sequence

import numpy as np

CACHE = os.path.expanduser(os.environ.get("PIERCE_AUTOTUNE_CACHE", "~/.cache/pierce_amd/autotune.json"))


def _digest(A, B, pairs) -> str:
    h = hashlib.sha256()
    for S in (A, B):
        h.update(np.ascontiguousarray(S.face_off).tobytes())
        h.update(np.ascontiguousarray(S.verts[:: max(1, S.verts.shape[0] // 4096)]).tobytes())
    h.update(np.ascontiguousarray(pairs).tobytes())
    return h.hexdigest()[:24]


def stratified_sample(A, B, pairs: np.ndarray, frac: float = 0.02, min_n: int = 256, n_buckets: int = 4,
                      seed: int = 0):
    """Indices of a seeded sample of `pairs`, the same fraction from each
    log-spaced bucket of F_A + F_B, and the bucket of every pair."""
    fa = np.diff(A.face_off)[pairs[:, 0]]
    fb = np.diff(B.face_off)[pairs[:, 1]]
    size = (fa + fb).astype(np.float64)
    edges = np.exp(np.linspace(np.log(size.min()), np.log(size.max() + 1), n_buckets + 1))
    bucket = np.clip(np.searchsorted(edges, size, side="right") - 1, 0, n_buckets - 1)
    rng = np.random.default_rng(seed)
    n = max(min_n, int(round(frac * pairs.shape[0])))
    idx = []
    for b in range(n_buckets):
        members = np.nonzero(bucket == b)[0]
        if members.size == 0:
            continue
        k = max(1, int(round(n * members.size / pairs.shape[0])))
        idx.append(rng.choice(members, size=min(k, members.size), replace=False))
    return np.sort(np.concatenate(idx)), bucket, edges


def _lib_digest() -> str:
    from . import _lib
    h = hashlib.sha256()
    with open(_lib.LIB_PATH, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


# Schedules swept: (schedule, per-bucket table of the automatic schedule).
# Tables: byte k = the largest number of a group's segments meeting the target
# box for which the group goes wave-per-segment, for targets below 2^10,
# 2^13, 2^16 triangles and larger.
def _schedule_grid(schedules, width):
    ns = 64 // width
    out = []
    for sc in schedules:
        if sc == 0:
            for t in (ns // 4, ns):
                t = max(1, t)
                out.append((0, t | (t << 8) | (t << 16) | (t << 24)))
        else:
            out.append((sc, 0))
    return out


def _time_refine(pa, torch, ga, gb, pairs_dev, cfg, reps: int) -> float:
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ws = pa.refine_workspace(int(pairs_dev.shape[0]), ga.width, cfg)
    flags = torch.empty(max(1, int(pairs_dev.shape[0])), dtype=torch.uint8, device="cuda")
    pa.refine(ga, gb, pairs_dev, cfg, ws=ws, flags=flags)  # warm-up
    ts = []
    for _ in range(reps):
        e0.record()
        pa.refine(ga, gb, pairs_dev, cfg, ws=ws, flags=flags)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(A, B, pairs, widths: Sequence[int] = (2, 4, 8), leaves: Sequence[int] = (1, 2, 4, 8),
         schedules: Sequence[int] = (0, 1, 2), frac: float = 0.02, n_buckets: int = 4, reps: int = 3,
         seed: int = 0, use_cache: bool = True, log=None, prefer=None, margin: float = 0.03) -> Dict:
    """Returns {"best": {"width", "leaf_size", "schedule", "seg_live_max", "ms"}, "table": [...],
    "per_bucket": {bucket: best config}, "sample": n}.  prefer = (width, leaf_size, schedule): that
    configuration stays the best unless another is faster by more than `margin` (a fraction),
    so that timing noise (about 2% between runs) does not flip the choice."""
    import torch
    import paper_2609_24513_amd as pa

    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    key = "%s|%s|%s|%s|%s|%s|%.4f|%d|%s|%.3f" % (torch.cuda.get_device_name(0), _lib_digest(), _digest(A, B, pairs),
                                                tuple(widths), tuple(leaves), tuple(schedules), frac, n_buckets,
                                                prefer, margin)
    if use_cache and os.path.exists(CACHE):
        try:
            cached = json.load(open(CACHE)).get(key)
            if cached:
                cached["cached"] = True
                return cached
        except (OSError, ValueError):
            pass
    idx, bucket, edges = stratified_sample(A, B, pairs, frac=frac, n_buckets=n_buckets, seed=seed)
    sample = torch.as_tensor(pairs[idx]).cuda()
    per_bucket_pairs = {int(b): torch.as_tensor(pairs[idx[bucket[idx] == b]]).cuda()
                        for b in np.unique(bucket[idx])}
    table = []
    t0 = time.perf_counter()
    for W in widths:
        for L in leaves:
            ga = pa.MeshBlob.build(A, width=W, leaf_size=L)
            gb = pa.MeshBlob.build(B, width=W, leaf_size=L)
            for sch, tab in _schedule_grid(schedules, W):
                cfg = pa.RefineConfig(persistent=1, schedule=sch, seg_live_max=tab)
                ms = _time_refine(pa, torch, ga, gb, sample, cfg, reps)
                row = {"width": W, "leaf_size": L, "schedule": sch, "seg_live_max": tab, "ms": ms, "buckets": {}}
                for b, pb in per_bucket_pairs.items():
                    row["buckets"][str(b)] = _time_refine(pa, torch, ga, gb, pb, cfg, reps)
                table.append(row)
                if log:
                    log("autotune W=%d L=%d schedule=%d table=%08x: %.3f ms on %d sampled pairs"
                        % (W, L, sch, tab, ms, len(idx)))
            del ga, gb
            torch.cuda.empty_cache()
    best = min(table, key=lambda r: r["ms"])
    if prefer is not None:
        pref = [r for r in table if (r["width"], r["leaf_size"], r["schedule"]) == tuple(prefer)]
        if pref and pref[0]["ms"] <= best["ms"] * (1.0 + margin):
            best = pref[0]
    per_bucket = {}
    for b in per_bucket_pairs:
        r = min(table, key=lambda r: r["buckets"][str(b)])
        per_bucket[str(b)] = {"width": r["width"], "leaf_size": r["leaf_size"], "schedule": r["schedule"],
                              "seg_live_max": r["seg_live_max"],
                              "ms": r["buckets"][str(b)], "size_range": [float(edges[b]), float(edges[b + 1])],
                              "pairs": int((bucket[idx] == b).sum())}
    out = {"best": {k: best[k] for k in ("width", "leaf_size", "schedule", "seg_live_max", "ms")}, "table": table,
           "per_bucket": per_bucket, "sample": int(len(idx)), "tune_seconds": time.perf_counter() - t0,
           "cached": False}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            data = json.load(open(CACHE)) if os.path.exists(CACHE) else {}
            data[key] = out
            json.dump(data, open(CACHE, "w"))
        except (OSError, ValueError):
            pass
    return out
