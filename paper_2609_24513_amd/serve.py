"""Serving loop: continuous batching of join queries over resident meshes.

A request is a query box; its answer is every pair (r, s) of the two resident
datasets whose closed mesh boxes meet each other and the query box and whose
surfaces share a point.  The loop keeps both datasets' BVH blobs in HBM and
runs without blocking the host:

  * arrivals go to a FIFO;
  * a slot is a HIP stream with its own device buffers (candidate regions,
    the gathered batch, flags, filter and refine workspaces), all allocated
    when the server starts; the HBM budget is spent on slots: the server
    opens as many slots as the budget holds (at least one, at most `slots`),
    so the device memory of the batches in flight never exceeds the budget
    (beyond the one slot every server needs);
  * a batch is opened whenever a slot is free: it admits up to
    max_req_per_batch waiting requests in arrival order (nothing waits while
    a slot is free, nothing is dropped);
  * the batch's query boxes go to the device in one asynchronous copy; each
    admitted request's candidate filter writes its own region of the slot,
    the regions are concatenated on the device with the counts left there
    (gather_pair_regions), and the concatenation is refined in ONE persistent
    launch that reads the count on the device: the whole batch is enqueued at
    once, with no host round trip; this work is captured once per slot and
    batch size as a HIP graph when the server starts, so a batch is one
    graph launch;
  * the counts, the status and the batch's pairs and flags (up to
    max_pairs per admitted request, an upper bound of the batch size) go
    back to pinned host buffers by asynchronous copies enqueued behind the
    refinement; when the slot's stream has finished, the results are read
    from those buffers with no further device transfer; a request completes
    then, and its latency is completion time minus arrival time.

Batches on different slots overlap on the device, and new requests are
admitted while earlier ones are still running.  The loop never sleeps: it
spins on arrivals and completions.  The per-request plain path
(`run_plain`) serves the same trace first-in first-out, one request at a
time, with one refinement launch per candidate pair.
"""
from __future__ import annotations

import ctypes
import dataclasses
import copy
import time
from collections import deque
from typing import List, Optional, Sequence

import numpy as np

from . import _lib

__all__ = ["Request", "JoinServer", "make_trace", "run_plain", "latency_summary"]


@dataclasses.dataclass
class Request:
    rid: int
    t_arrival: float            # seconds from the start of the trace
    box: np.ndarray             # f32[6] query box
    t_done: float = -1.0
    pairs: Optional[np.ndarray] = None   # int32[n, 2]
    flags: Optional[np.ndarray] = None   # uint8[n]

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def make_trace(box_r: np.ndarray, box_s: np.ndarray, n: int, lam: float, seed: int = 5,
               k_lo: float = 1.0, k_hi: float = 5000.0, space: float = 58.5, min_pairs: int = 1,
               max_pairs: int = 5000) -> List[Request]:
    """Requests of the seeded serving trace (synth.c5_queries): Poisson
    arrivals at rate lam, query boxes selecting min_pairs..max_pairs
    candidate pairs."""
    from . import synth
    q = synth.c5_queries(box_r, box_s, n, lam, seed=seed, k_lo=k_lo, k_hi=k_hi, space=space,
                         min_pairs=min_pairs, max_pairs=max_pairs)
    return [Request(rid, t, box) for rid, (t, box) in enumerate(q)]


def latency_summary(reqs: Sequence[Request]) -> dict:
    lat = np.array([r.latency for r in reqs]) * 1e3
    pairs = int(sum(0 if r.pairs is None else r.pairs.shape[0] for r in reqs))
    span = max(r.t_done for r in reqs) - min(r.t_arrival for r in reqs)
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "pairs": pairs,
            "pairs_per_s": pairs / span if span > 0 else 0.0, "span_s": span}


class _Slot:
    def __init__(self, torch, pa, R, S, max_req: int, max_pairs: int, cfg):
        self.torch = torch
        self.stream = torch.cuda.Stream()
        cap = max_req * max_pairs
        self.region = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
        self.counts = torch.zeros(max_req, dtype=torch.int64, device="cuda")
        self.counts_h = torch.zeros(max_req, dtype=torch.int64, pin_memory=True)
        self.batch = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
        self.flags = torch.empty(cap, dtype=torch.uint8, device="cuda")
        self.flags_h = torch.zeros(cap, dtype=torch.uint8, pin_memory=True)
        self.batch_h = torch.zeros((cap, 2), dtype=torch.int32, pin_memory=True)
        self.status = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.status_h = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        self.total = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.stats = torch.zeros(len(pa.STATS_FIELDS), dtype=torch.int64, device="cuda")
        self.graphs = {}        # batch size -> captured HIP graph of the batch's device work
        # query boxes of a batch: filled on the host, one asynchronous copy
        self.boxes_h = torch.zeros((max_req, 6), dtype=torch.float32, pin_memory=True)
        self.boxes = torch.empty((max_req, 6), dtype=torch.float32, device="cuda")
        lib = _lib.load()
        wb = ctypes.c_size_t(0)
        _lib.check(lib.filter_aabb_pairs_ws_bytes(R.n_meshes, S.n_meshes, ctypes.byref(wb)))
        self.fws = torch.empty(max(256, wb.value), dtype=torch.uint8, device="cuda")
        self.rws = pa.refine_workspace(cap, R.width, cfg)
        self.reqs: List[Request] = []
        self.phase = 0          # 0 free, 1 on the device
        self.event = None

    def bytes(self) -> int:
        t = [self.region, self.counts, self.batch, self.flags, self.fws, self.rws, self.boxes, self.status,
             self.total]
        return int(sum(x.numel() * x.element_size() for x in t))


class JoinServer:
    """Continuous-batching server over two resident MeshBlobs (see module doc)."""

    def __init__(self, R, S, max_req_per_batch: int = 32, max_pairs: int = 5000, slots: int = 3,
                 hbm_budget: int = 1 << 30, cfg=None, graphs: bool = True):
        import torch
        import paper_2609_24513_amd as pa
        self.torch, self.pa = torch, pa
        self.R, self.S = R, S
        self.max_pairs = max_pairs
        self.max_req = max_req_per_batch
        self.cfg = cfg or pa.RefineConfig(persistent=1)
        if self.cfg.survivor_cap == 0:
            # a batch queues at most (groups of the largest mesh of R + of S) per pair
            gmax = int((R.edge_counts().max().item() + 63) // 64 + (S.edge_counts().max().item() + 63) // 64)
            cfg2 = copy.copy(self.cfg)
            cfg2.survivor_cap = int(min(1 << 24, max(1 << 16, gmax * max_req_per_batch * max_pairs)))
            self.cfg = cfg2
        self.hbm_budget = int(hbm_budget)
        first = _Slot(torch, pa, R, S, max_req_per_batch, max_pairs, self.cfg)
        self.slot_bytes = first.bytes()
        n_slots = int(min(max(1, slots), max(1, self.hbm_budget // max(1, self.slot_bytes))))
        self.slots = [first] + [_Slot(torch, pa, R, S, max_req_per_batch, max_pairs, self.cfg)
                                for _ in range(n_slots - 1)]
        self.in_flight_bytes = 0      # device bytes of the slots with a batch in flight
        self.batches = 0
        self.max_in_flight = 0
        self.oversized = 0      # requests beyond max_pairs, answered on their own
        self._t0 = None
        self.graphs = graphs and self._capture()

    # --- phases ------------------------------------------------------------
    def _enqueue(self, slot: _Slot, n: int):
        """The device work of a batch of n requests whose query boxes are in
        slot.boxes_h[:n], on the slot's stream with no host round trip: the
        boxes copied in, one filter per query into its region, the regions
        concatenated on the device (gather_pair_regions), one refinement of
        the concatenation with the device count, then the counts, status,
        pairs and flags copied back to pinned host buffers.  Every buffer
        is the slot's own, so the same work can be captured once per batch
        size and replayed."""
        torch, pa, lib = self.torch, self.pa, _lib.load()
        cap = slot.batch.shape[0]
        with torch.cuda.stream(slot.stream):
            sp = int(slot.stream.cuda_stream)
            slot.boxes[:n].copy_(slot.boxes_h[:n], non_blocking=True)
            for k in range(n):
                _lib.check(lib.filter_aabb_pairs(
                    self.R.ptr, self.R.n_meshes, self.S.ptr, self.S.n_meshes, slot.boxes.data_ptr() + 24 * k,
                    slot.region.data_ptr() + k * self.max_pairs * 8, self.max_pairs,
                    slot.counts.data_ptr() + 8 * k, slot.fws.data_ptr(), slot.fws.numel(), sp))
            _lib.check(lib.gather_pair_regions(slot.region.data_ptr(), self.max_pairs, slot.counts.data_ptr(),
                                               n, slot.batch.data_ptr(), cap, slot.total.data_ptr(), sp))
            cfg = copy.copy(self.cfg)
            cfg.n_dev = slot.total
            # a batch of n requests holds at most n * max_pairs pairs: the
            # launch is sized for that many (small batches skip the cull order)
            pa.refine(self.R, self.S, slot.batch[:n * self.max_pairs], cfg, ws=slot.rws, flags=slot.flags,
                      stats=slot.stats, status=slot.status, stream=slot.stream)
            slot.counts_h[:n].copy_(slot.counts[:n], non_blocking=True)
            slot.status_h.copy_(slot.status, non_blocking=True)
            # every request holds at most max_pairs candidates in the batch
            m = n * self.max_pairs
            slot.batch_h[:m].copy_(slot.batch[:m], non_blocking=True)
            slot.flags_h[:m].copy_(slot.flags[:m], non_blocking=True)

    def _capture(self) -> bool:
        """Captures each slot's batch work for every batch size (HIP graphs:
        one launch per batch instead of one per kernel and copy).  A batch of
        each slot runs eagerly first, so that the library's per-device
        queries are cached outside the capture.  Returns False (eager
        batches) if the runtime refuses a capture."""
        torch = self.torch
        for slot in self.slots:
            slot.boxes_h[0] = 3e38  # a point far outside every mesh box: no candidates
            self._enqueue(slot, 1)
        torch.cuda.synchronize()
        try:
            for slot in self.slots:
                for n in range(1, self.max_req + 1):
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=slot.stream, capture_error_mode="thread_local"):
                        self._enqueue(slot, n)
                    slot.graphs[n] = g
        except RuntimeError:
            torch.cuda.synchronize()
            for slot in self.slots:
                slot.graphs = {}
            return False
        torch.cuda.synchronize()
        return True

    def _start(self, slot: _Slot, reqs: List[Request]):
        """Enqueues the whole batch on the slot's stream: its captured graph
        (or the same work eagerly), then the completion event."""
        torch = self.torch
        slot.reqs = reqs
        slot.phase = 1
        # the slot is free, so its previous box copy has completed
        bh = slot.boxes_h.numpy()
        for k, r in enumerate(reqs):
            bh[k] = r.box
        n = len(reqs)
        with torch.cuda.stream(slot.stream):
            if self.graphs:
                slot.graphs[n].replay()
            else:
                self._enqueue(slot, n)
            slot.event = torch.cuda.Event()
            slot.event.record(slot.stream)

    def _finish(self, slot: _Slot, now: float):
        raw = slot.counts_h[:len(slot.reqs)].numpy().astype(np.int64)
        counts = np.minimum(np.maximum(raw, 0), self.max_pairs)
        offsets = np.concatenate([[0], np.cumsum(counts)])
        n = int(offsets[-1])
        if n and int(slot.status_h.item()) != 0:
            raise RuntimeError("refine status %d" % int(slot.status_h.item()))
        # copied out of the pinned buffers, which the slot's next batch reuses
        flags = slot.flags_h[:n].numpy().copy()
        pairs = slot.batch_h[:n].numpy().copy()
        for k, r in enumerate(slot.reqs):
            if raw[k] > self.max_pairs:
                # more candidates than a slot region holds: this request's
                # region was truncated, so it is answered again on its own
                # with a buffer of the exact size
                r.pairs, r.flags = self._serve_large(r.box, int(raw[k]))
                self.oversized += 1
                r.t_done = time.perf_counter() - self._t0
            else:
                a, b = int(offsets[k]), int(offsets[k + 1])
                r.pairs = pairs[a:b]
                r.flags = flags[a:b]
                r.t_done = now
        self.in_flight_bytes -= self.slot_bytes
        slot.reqs = []
        slot.phase = 0
        slot.event = None

    def _serve_large(self, box: np.ndarray, count: int):
        """A request whose candidate count exceeds max_pairs: filter with a
        buffer of exactly `count` pairs, then one refinement, synchronously."""
        pa, torch = self.pa, self.torch
        pairs = pa.filter_pairs(self.R, self.S, query_box=box, cap=count)
        flags, _, status = pa.refine(self.R, self.S, pairs, self.cfg)
        torch.cuda.synchronize()
        if int(status.item()) != 0:
            raise RuntimeError("refine status %d" % int(status.item()))
        return pairs.cpu().numpy(), flags.cpu().numpy()

    # --- loop ----------------------------------------------------------------
    def run(self, trace: Sequence[Request], realtime: bool = True) -> List[Request]:
        """Serves `trace` (requests sorted by arrival).  With realtime=True the
        requests are released at their arrival times on the host clock."""
        pending = deque()
        todo = deque(sorted(trace, key=lambda r: r.t_arrival))
        t0 = time.perf_counter()
        self._t0 = t0
        done = 0
        n = len(todo)
        while done < n:
            now = time.perf_counter() - t0
            while todo and (todo[0].t_arrival <= now or not realtime):
                r = todo.popleft()
                if not realtime:
                    r.t_arrival = now
                pending.append(r)
            progressed = False
            for slot in self.slots:
                if slot.phase and slot.event.query():
                    k = len(slot.reqs)
                    self._finish(slot, time.perf_counter() - t0)
                    done += k
                    progressed = True
            for slot in self.slots:
                if slot.phase == 0 and pending:
                    batch = []
                    while pending and len(batch) < self.max_req:
                        batch.append(pending.popleft())
                    if batch:
                        self.in_flight_bytes += self.slot_bytes
                        self._start(slot, batch)
                        self.batches += 1
                        progressed = True
                    busy = sum(1 for s in self.slots if s.phase)
                    self.max_in_flight = max(self.max_in_flight, busy)
            if not progressed:
                # the loop spins (yielding the interpreter lock each turn), so
                # that arrivals and completions are picked up at once: a timed
                # sleep would add its length and the timer slack to the
                # latency of a request arriving meanwhile
                time.sleep(0)
        return list(trace)

    def query_alone(self, box: np.ndarray):
        """One request on its own (filter with relaunch on overflow, then
        refine): (pairs, flags)."""
        pa, torch = self.pa, self.torch
        pairs = pa.filter_pairs(self.R, self.S, query_box=box, cap=self.max_pairs)
        if pairs.shape[0] == 0:
            return np.zeros((0, 2), np.int32), np.zeros(0, np.uint8)
        flags, _, status = pa.refine(self.R, self.S, pairs, self.cfg)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        return pairs.cpu().numpy(), flags.cpu().numpy()


def run_plain(R, S, trace: Sequence[Request], realtime: bool = True, max_pairs: int = 5000) -> List[Request]:
    """First-in first-out, one request at a time: filter, then one refinement
    launch per candidate pair, then the flags back to the host."""
    import torch
    import paper_2609_24513_amd as pa
    cfg = pa.RefineConfig(persistent=0)
    ws = pa.refine_workspace(max_pairs, R.width, cfg)
    reqs = sorted(trace, key=lambda r: r.t_arrival)
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0
        if realtime and now < r.t_arrival:
            time.sleep(r.t_arrival - now)
        pairs = pa.filter_pairs(R, S, query_box=r.box, cap=max_pairs)
        if pairs.shape[0]:
            flags, _, status = pa.refine(R, S, pairs, cfg, ws=ws)
            r.flags = flags.cpu().numpy()
            r.pairs = pairs.cpu().numpy()
        else:
            r.flags = np.zeros(0, np.uint8)
            r.pairs = np.zeros((0, 2), np.int32)
        r.t_done = time.perf_counter() - t0
    return list(trace)
