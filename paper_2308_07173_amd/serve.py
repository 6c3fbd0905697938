"""Continuous-batching request loop: LiDAR scans against resident target maps.

Several sensors stream scans (the paper's cars carry three LiDARs feeding one
PC; Sec. IV-B platform tables); every scan needs the nearest points and
covariances of its points in one of the device-resident maps (Sec. III-C.1,
III-C.3).  This module serves such a stream on one GPU:

* maps are built once and stay resident (one ``TargetSet``);
* requests are admitted FIFO into batches; the device memory the server may
  use (``hbm_budget_bytes``) fixes how many queries can be in flight, and a
  request waits while that budget is taken;
* two batch slots, each with its own HIP stream, library context, buffers
  and target-set table, so a new batch is assembled, uploaded and launched
  while the other is still running (their copies and kernels overlap);
* a batch is one ``lkc_knn_cov_batched`` call, optionally replayed from a
  HIP graph captured per padded batch size (padding rows are NaN queries,
  which the kernels answer with count 0);
* latency is measured from a request's arrival to the moment its batch's
  completion event is observed on the host.

The scheduling policy (``plan_batch``, ``serve_loop``) is plain Python and is
exercised on the CPU with a modelled executor.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class ServeRequest:
    rid: int
    t_arrival: float          # seconds from stream start (schedule time)
    map_id: int
    points: np.ndarray        # float32 [n, 3], world frame
    sensor: int = 0


def bytes_per_query(k: int) -> int:
    """Device bytes one in-flight query holds: the query, its outputs
    (idx, d2, count, mean, cov, reg_cov, valid) and the search scratch."""
    return 12 + 8 * k + 4 + 12 + 36 + 36 + 1 + 36


def plan_batch(pending: collections.deque, capacity: int) -> List[ServeRequest]:
    """Take requests FIFO while they fit in `capacity` queries (a request
    never overtakes an earlier one that does not fit)."""
    batch: List[ServeRequest] = []
    used = 0
    while pending:
        n = pending[0].points.shape[0]
        if used + n > capacity:
            break
        batch.append(pending.popleft())
        used += n
    return batch


class Executor:
    """Interface of a batch executor with `n_slots` independent slots."""
    n_slots: int
    capacity: int             # queries per slot

    def launch(self, slot: int, batch: List[ServeRequest]) -> None: ...

    def poll(self, slot: int) -> bool:
        """True once the batch launched on `slot` has finished."""
        ...

    def finish(self, slot: int, batch: List[ServeRequest]) -> None:
        """Called once per completed batch (results may be collected here)."""


def serve_loop(requests: Sequence[ServeRequest], ex: Executor, time_scale: float = 1.0,
               clock: Callable[[], float] = time.perf_counter,
               idle: Callable[[], None] = lambda: None) -> Dict:
    """Replay `requests` (sorted by arrival) against `ex`.

    time_scale compresses the schedule (arrival t is released at t /
    time_scale); math.inf releases everything at once (open loop).
    Returns per-request latencies (s) and the wall time.
    """
    reqs = sorted(requests, key=lambda r: (r.t_arrival, r.rid))
    for r in reqs:
        if r.points.shape[0] > ex.capacity:
            raise ValueError(f"request {r.rid} ({r.points.shape[0]} points) exceeds the "
                             f"batch capacity {ex.capacity}")
    t0 = clock()
    pending: collections.deque = collections.deque()
    inflight: List[Optional[List[ServeRequest]]] = [None] * ex.n_slots
    release = {}
    latency = {}
    batches = []
    nxt = 0
    done = 0
    while done < len(reqs):
        now = clock() - t0
        progressed = False
        while nxt < len(reqs):
            r = reqs[nxt]
            rel = 0.0 if math.isinf(time_scale) else r.t_arrival / time_scale
            if rel > now:
                break
            pending.append(r)
            release[r.rid] = rel
            nxt += 1
            progressed = True
        for s in range(ex.n_slots):
            b = inflight[s]
            if b is not None and ex.poll(s):
                t_done = clock() - t0
                for r in b:
                    latency[r.rid] = t_done - release[r.rid]
                ex.finish(s, b)
                inflight[s] = None
                done += len(b)
                progressed = True
        for s in range(ex.n_slots):
            if inflight[s] is None and pending:
                b = plan_batch(pending, ex.capacity)
                if b:
                    ex.launch(s, b)
                    inflight[s] = b
                    batches.append(len(b))
                    progressed = True
        if not progressed:
            idle()
    wall = clock() - t0
    lat = np.array([latency[r.rid] for r in reqs])
    nq = int(sum(r.points.shape[0] for r in reqs))
    return {"latency_s": lat, "wall_s": wall, "queries": nq, "requests": len(reqs),
            "batches": len(batches), "mean_batch_requests": float(np.mean(batches)) if batches else 0.0}


def summarize(res: Dict) -> Dict:
    lat = res["latency_s"]
    return {"queries_per_s": res["queries"] / res["wall_s"],
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "max_ms": float(lat.max() * 1e3), "requests": res["requests"],
            "batches": res["batches"], "mean_batch_requests": res["mean_batch_requests"],
            "wall_s": res["wall_s"]}


# ------------------------------------------------------------- GPU side --

class GpuExecutor(Executor):
    """Two-slot executor over lkc_knn_cov_batched on resident targets."""

    BUCKETS = (1 << 15, 1 << 16, 1 << 17, 1 << 18, 1 << 19, 1 << 20, 1 << 21, 1 << 22)

    def __init__(self, targets_points: Sequence[np.ndarray], cell: float = 1.0, k: int = 20,
                 radius: float = 2.0, eps: float = 1e-3, hbm_budget_bytes: Optional[int] = None,
                 n_slots: int = 2, use_graphs: bool = True, max_scans: int = 256,
                 keep_results: bool = False, cfg=None):
        import torch
        from paper_2308_07173_amd import lkc
        self.torch, self.lkc = torch, lkc
        self.k, self.radius, self.eps, self.cfg = k, radius, eps, cfg
        self.n_slots = n_slots
        self.keep_results = keep_results
        self.results: Dict[int, Dict[str, np.ndarray]] = {}
        self.dev = torch.device("cuda", torch.cuda.current_device())
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget_bytes = int(0.8 * free)
        self.budget = int(hbm_budget_bytes)
        # resident maps: built once on a set-up context, counted against the
        # budget before any request
        self.setup_ctx = lkc.Context()
        self.map_dev = [torch.from_numpy(np.ascontiguousarray(p)).to(self.dev)
                        for p in targets_points]
        self.targets = [lkc.lkc_build_target(self.setup_ctx, m, cell) for m in self.map_dev]
        torch.cuda.synchronize()
        self.resident_bytes = int(sum(t.info()["device_bytes"] for t in self.targets) +
                                  sum(m.numel() * 4 for m in self.map_dev))
        per_q = bytes_per_query(k)
        cap = (self.budget - self.resident_bytes) // (n_slots * per_q)
        cap = min(cap, self.BUCKETS[-1])
        if cap < 1:
            raise ValueError("HBM budget too small for one query beside the resident maps")
        self.capacity = int(cap)
        self.use_graphs = use_graphs
        # resident maps: built once on a set-up context
        self.setup_ctx = lkc.Context()
        self.map_dev = [torch.from_numpy(np.ascontiguousarray(p)).to(self.dev)
                        for p in targets_points]
        self.targets = [lkc.lkc_build_target(self.setup_ctx, m, cell) for m in self.map_dev]
        torch.cuda.synchronize()
        self.slots = []
        for _ in range(n_slots):
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                ctx = lkc.Context()
                ctx.reserve(self.capacity)
                tset = lkc.TargetSet(ctx, self.targets, max_scans)
            q_host = torch.empty((self.capacity, 3), dtype=torch.float32, pin_memory=True)
            q_dev = torch.empty((self.capacity, 3), dtype=torch.float32, device=self.dev)
            out = dict(idx=torch.empty((self.capacity, k), dtype=torch.int32, device=self.dev),
                       d2=torch.empty((self.capacity, k), dtype=torch.float32, device=self.dev),
                       count=torch.empty(self.capacity, dtype=torch.int32, device=self.dev),
                       mean=torch.empty((self.capacity, 3), dtype=torch.float32, device=self.dev),
                       cov=torch.empty((self.capacity, 3, 3), dtype=torch.float32, device=self.dev),
                       reg=torch.empty((self.capacity, 3, 3), dtype=torch.float32, device=self.dev),
                       valid=torch.empty(self.capacity, dtype=torch.uint8, device=self.dev))
            self.slots.append(dict(stream=st, ctx=ctx, tset=tset, q_host=q_host, q_dev=q_dev,
                                   out=out, done=torch.cuda.Event(), graphs={}, n=0,
                                   offsets=None))
        self.max_scans = max_scans

    def _bucket(self, n: int) -> int:
        for b in self.BUCKETS:
            if b >= n and b <= self.capacity:
                return b
        return self.capacity

    def _call(self, s, total):
        lkc = self.lkc
        views = {key: v[:total] for key, v in s["out"].items()}
        lkc.lkc_knn_cov_batched(s["ctx"], s["tset"], s["q_dev"][:total], self.k, self.radius,
                                self.eps, out=views, cfg=self.cfg)

    def launch(self, slot: int, batch: List[ServeRequest]) -> None:
        torch = self.torch
        s = self.slots[slot]
        sizes = [r.points.shape[0] for r in batch]
        n = int(sum(sizes))
        total = self._bucket(n) if self.use_graphs else n
        qh = s["q_host"].numpy()
        off = 0
        scans = []
        for r, m in zip(batch, sizes):
            qh[off:off + m] = r.points
            scans.append((off, m, r.map_id))
            off += m
        if total > n:
            scans.append((n, total - n, 0))
        if len(scans) > self.max_scans:
            raise ValueError("too many scans in one batch")
        with torch.cuda.stream(s["stream"]):
            s["q_dev"][:n].copy_(s["q_host"][:n], non_blocking=True)
            if total > n:
                s["q_dev"][n:total].fill_(float("nan"))
            s["tset"].stage(scans)
            if self.use_graphs:
                g = s["graphs"].get(total)
                if g is None:
                    self._call(s, total)          # warm-up outside the capture
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=s["stream"]):
                        self._call(s, total)
                    s["graphs"][total] = g
                g.replay()
            else:
                self._call(s, total)
            s["done"].record(s["stream"])
        s["n"] = n
        s["offsets"] = np.cumsum([0] + sizes)

    def poll(self, slot: int) -> bool:
        return self.slots[slot]["done"].query()

    def finish(self, slot: int, batch: List[ServeRequest]) -> None:
        if not self.keep_results:
            return
        s = self.slots[slot]
        offs = s["offsets"]
        host = {key: v[:s["n"]].cpu().numpy() for key, v in s["out"].items()}
        for i, r in enumerate(batch):
            self.results[r.rid] = {key: v[offs[i]:offs[i + 1]].copy() for key, v in host.items()}

    def close(self):
        self.torch.cuda.synchronize()
        for s in self.slots:
            s["graphs"].clear()
            s["tset"].free()
            s["ctx"].close()
        for t in self.targets:
            t.free()
        self.setup_ctx.close()


def plain_loop(requests: Sequence[ServeRequest], ex: GpuExecutor, time_scale: float = 1.0) -> Dict:
    """Reference path: each request is searched alone (one lkc_knn_cov call on
    one stream) in arrival order, as soon as it has arrived and the previous
    one is done."""
    torch, lkc = ex.torch, ex.lkc
    reqs = sorted(requests, key=lambda r: (r.t_arrival, r.rid))
    ctx = lkc.Context()
    ctx.reserve(max(r.points.shape[0] for r in reqs))
    t0 = time.perf_counter()
    lat = []
    for r in reqs:
        rel = 0.0 if math.isinf(time_scale) else r.t_arrival / time_scale
        while time.perf_counter() - t0 < rel:
            pass
        q = torch.from_numpy(r.points).to(ex.dev, non_blocking=False)
        lkc.lkc_knn_cov(ctx, ex.targets[r.map_id], q, ex.k, ex.radius, ex.eps, cfg=ex.cfg)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - rel)
    wall = time.perf_counter() - t0
    ctx.close()
    return {"latency_s": np.array(lat), "wall_s": wall,
            "queries": int(sum(r.points.shape[0] for r in reqs)), "requests": len(reqs),
            "batches": len(reqs), "mean_batch_requests": 1.0}
