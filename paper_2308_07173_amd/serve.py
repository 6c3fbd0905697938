"""Continuous-batching request loop: LiDAR scans against resident target maps.

Several sensors stream scans (the paper's cars carry three LiDARs feeding one
PC; Sec. IV-B platform tables); every scan needs the nearest points and
covariances of its points in one of the device-resident maps (Sec. III-C.1,
III-C.3).  This module serves such a stream on one GPU:

* maps are built once and stay resident; their bytes are counted against
  the device-memory budget (``hbm_budget_bytes``), and maps can be added or
  removed between streams;
* requests are admitted FIFO into batches.  Each batch claims the device
  bytes of its own buffers (query + outputs per padded row) from what the
  budget leaves beside the resident maps and the slots' fixed search
  scratch; a batch that does not fit waits (the request is *deferred*) until
  running batches release their bytes, and is admitted then;
* every request ends with a status: ``done``, ``unknown_map`` (its map id is
  not resident), ``over_budget`` (it cannot fit even with nothing else in
  flight) or ``cancelled`` (cancelled before its batch was launched); a
  failed request never stops the others;
* two batch slots, each with its own HIP stream, library context and
  target-set table, so a new batch is assembled, uploaded and launched while
  the other is still running;
* a batch is one ``lkc_knn_cov_batched`` call, optionally replayed from a
  HIP graph captured per buffer set; buffer sets come in row buckets at most
  12.5 % above the batch (padding rows are NaN queries, which the kernels
  answer with count 0);
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
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

DONE = "done"
UNKNOWN_MAP = "unknown_map"
OVER_BUDGET = "over_budget"
CANCELLED = "cancelled"


@dataclasses.dataclass(eq=False)
class ServeRequest:
    rid: int
    t_arrival: float          # seconds from stream start (schedule time)
    map_id: int
    points: np.ndarray        # float32 [n, 3], world frame
    sensor: int = 0


# Search scratch the library holds per query of a context's largest call
# (sort keys and values twice, fallback list, 25 % headroom).
SCRATCH_BYTES_PER_QUERY = 36


def row_bytes(k: int) -> int:
    """Device bytes of one batch row: the query and its outputs (idx, d2,
    count, mean, cov, reg_cov, valid)."""
    return 12 + 8 * k + 4 + 12 + 36 + 36 + 1


def bytes_per_query(k: int) -> int:
    """Device bytes one in-flight query holds: its row and its share of the
    search scratch."""
    return row_bytes(k) + SCRATCH_BYTES_PER_QUERY


def bucket_rows(n: int, min_rows: int = 1024) -> int:
    """Rows of the buffer set for a batch of n queries: n rounded up to a
    multiple of 2^(floor(log2 n) - 3) (at most 12.5 % padding), and at least
    min_rows."""
    if n <= min_rows:
        return min_rows
    step = 1 << max(0, n.bit_length() - 1 - 3)
    return -(-n // step) * step


def plan_batch(pending: collections.deque, capacity: int,
               max_requests: Optional[int] = None) -> List[ServeRequest]:
    """Take requests FIFO while they fit in `capacity` queries and
    `max_requests` requests (a request never overtakes an earlier one that
    does not fit)."""
    batch: List[ServeRequest] = []
    used = 0
    while pending and (max_requests is None or len(batch) < max_requests):
        n = pending[0].points.shape[0]
        if used + n > capacity:
            break
        batch.append(pending.popleft())
        used += n
    return batch


class Executor:
    """Interface of a batch executor with `n_slots` independent slots."""
    n_slots: int
    capacity: int             # queries per batch
    max_batch_requests: Optional[int] = None

    def has_map(self, map_id: int) -> bool:
        return True

    def max_request_queries(self) -> int:
        """The largest request that fits with nothing else in flight."""
        return self.capacity

    def reserve(self, slot: int, batch: List[ServeRequest]) -> bool:
        """Claim the device bytes of `batch` for `slot`; False when the
        budget cannot hold them now (nothing is claimed then)."""
        return True

    def launch(self, slot: int, batch: List[ServeRequest]) -> None: ...

    def poll(self, slot: int) -> bool:
        """True once the batch launched on `slot` has finished."""
        ...

    def finish(self, slot: int, batch: List[ServeRequest]) -> None:
        """Called once per completed batch (releases its bytes; results may
        be collected here)."""

    def memory(self) -> Dict[str, int]:
        return {}


def serve_loop(requests: Sequence[ServeRequest], ex: Executor, time_scale: float = 1.0,
               clock: Callable[[], float] = time.perf_counter,
               idle: Callable[[], None] = lambda: None,
               cancels: Iterable[Tuple[float, int]] = ()) -> Dict:
    """Replay `requests` (sorted by arrival) against `ex`.

    time_scale compresses the schedule (arrival t is released at t /
    time_scale); math.inf releases everything at once (open loop).
    cancels: (schedule time, rid) pairs; a request still queued (or not yet
    arrived) at that time is dropped with status ``cancelled``; one already
    launched completes.
    Returns per-request statuses, the latencies of the completed requests
    (s, in request order), admission counters and the wall time.
    """
    reqs = sorted(requests, key=lambda r: (r.t_arrival, r.rid))
    by_rid = {r.rid: r for r in reqs}
    cancel_q = collections.deque(sorted(cancels))
    t0 = clock()
    pending: collections.deque = collections.deque()
    inflight: List[Optional[List[ServeRequest]]] = [None] * ex.n_slots
    status: Dict[int, str] = {}
    cancelled_early = set()
    release = {}
    latency = {}
    deferred = set()
    batches = []
    late_cancels = 0
    max_inflight_bytes = 0
    nxt = 0

    def rel_time(t):
        return 0.0 if math.isinf(time_scale) else t / time_scale

    while len(status) < len(reqs):
        now = clock() - t0
        progressed = False
        # arrivals
        while nxt < len(reqs):
            r = reqs[nxt]
            rel = rel_time(r.t_arrival)
            if rel > now:
                break
            nxt += 1
            progressed = True
            release[r.rid] = rel
            if r.rid in cancelled_early:
                status[r.rid] = CANCELLED
            elif not ex.has_map(r.map_id):
                status[r.rid] = UNKNOWN_MAP
            elif r.points.shape[0] > ex.max_request_queries():
                status[r.rid] = OVER_BUDGET
            else:
                pending.append(r)
        # cancellations due by now
        while cancel_q and rel_time(cancel_q[0][0]) <= now:
            _, rid = cancel_q.popleft()
            progressed = True
            if rid not in by_rid:
                continue
            if rid in status:
                if status[rid] == DONE:
                    late_cancels += 1
                continue
            r = by_rid[rid]
            if r in pending:
                pending.remove(r)
                status[rid] = CANCELLED
            elif rid not in release:
                cancelled_early.add(rid)
            else:
                late_cancels += 1          # already launched: it completes
        # completions
        for s in range(ex.n_slots):
            b = inflight[s]
            if b is not None and ex.poll(s):
                t_done = clock() - t0
                for r in b:
                    latency[r.rid] = t_done - release[r.rid]
                    status[r.rid] = DONE
                ex.finish(s, b)
                inflight[s] = None
                progressed = True
        # admissions
        for s in range(ex.n_slots):
            if inflight[s] is not None or not pending:
                continue
            b = plan_batch(pending, ex.capacity, ex.max_batch_requests)
            if b and not ex.reserve(s, b):
                # over the budget now: the batch waits at the head of the queue
                for r in reversed(b):
                    pending.appendleft(r)
                deferred.update(r.rid for r in b)
                if any(x is not None for x in inflight):
                    break                  # running batches will release bytes
                # nothing in flight: the head alone, else it can never fit
                b = [pending.popleft()]
                if not ex.reserve(s, b):
                    status[b[0].rid] = OVER_BUDGET
                    progressed = True
                    continue
            if b:
                ex.launch(s, b)
                inflight[s] = b
                batches.append(len(b))
                progressed = True
                mem = ex.memory()
                if mem:
                    max_inflight_bytes = max(max_inflight_bytes, mem.get("inflight", 0))
        if not progressed:
            idle()
    wall = clock() - t0
    done = [r for r in reqs if status[r.rid] == DONE]
    lat = np.array([latency[r.rid] for r in done])
    nq = int(sum(r.points.shape[0] for r in done))
    counts = collections.Counter(status.values())
    return {"latency_s": lat, "wall_s": wall, "queries": nq, "requests": len(reqs),
            "completed": len(done), "status": status,
            "status_counts": {k: counts.get(k, 0) for k in (DONE, UNKNOWN_MAP, OVER_BUDGET,
                                                           CANCELLED)},
            "deferred": len(deferred), "late_cancels": int(late_cancels),
            "max_inflight_bytes": int(max_inflight_bytes),
            "batches": len(batches),
            "mean_batch_requests": float(np.mean(batches)) if batches else 0.0}


def summarize(res: Dict) -> Dict:
    lat = res["latency_s"]
    have = len(lat) > 0
    return {"queries_per_s": res["queries"] / res["wall_s"] if res["wall_s"] > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if have else float("nan"),
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if have else float("nan"),
            "max_ms": float(lat.max() * 1e3) if have else float("nan"),
            "requests": res["requests"], "completed": res["completed"],
            "status_counts": res["status_counts"], "deferred": res["deferred"],
            "batches": res["batches"], "mean_batch_requests": res["mean_batch_requests"],
            "wall_s": res["wall_s"]}


# ------------------------------------------------------------- GPU side --

class _BufferSet:
    """Device buffers of one batch of up to `rows` queries, and the graphs
    captured on them (one per slot)."""

    def __init__(self, torch, dev, rows: int, k: int):
        self.rows = rows
        self.q_dev = torch.empty((rows, 3), dtype=torch.float32, device=dev)
        self.out = dict(idx=torch.empty((rows, k), dtype=torch.int32, device=dev),
                        d2=torch.empty((rows, k), dtype=torch.float32, device=dev),
                        count=torch.empty(rows, dtype=torch.int32, device=dev),
                        mean=torch.empty((rows, 3), dtype=torch.float32, device=dev),
                        cov=torch.empty((rows, 3, 3), dtype=torch.float32, device=dev),
                        reg=torch.empty((rows, 3, 3), dtype=torch.float32, device=dev),
                        valid=torch.empty(rows, dtype=torch.uint8, device=dev))
        self.graphs: Dict[int, object] = {}


class GpuExecutor(Executor):
    """Two-slot executor over lkc_knn_cov_batched on resident targets.

    Device bytes: resident maps (their targets) + the slots' search scratch
    (fixed, for `capacity` queries each) + the buffer sets (rows x row_bytes),
    all within `hbm_budget_bytes`.  Buffer sets are kept per row bucket for
    reuse (and their graphs with them) and evicted when a new set needs
    their bytes."""

    MAX_ROWS = 1 << 22

    def __init__(self, targets_points: Sequence[np.ndarray], cell: float = 1.0, k: int = 20,
                 radius: float = 2.0, eps: float = 1e-3, hbm_budget_bytes: Optional[int] = None,
                 n_slots: int = 2, use_graphs: bool = True, max_scans: int = 256,
                 keep_results: bool = False, cfg=None, max_rows: int = MAX_ROWS):
        import torch
        from paper_2308_07173_amd import lkc
        self.torch, self.lkc = torch, lkc
        self.k, self.radius, self.eps, self.cfg, self.cell = k, radius, eps, cfg, cell
        self.n_slots = n_slots
        self.keep_results = keep_results
        self.use_graphs = use_graphs
        # capture a graph for a buffer set the first time it runs; off, a
        # set without one runs eagerly (no capture latency inside a stream)
        self.capture_new = True
        self.max_scans = max_scans
        self.max_batch_requests = max_scans - 1      # one table row for the padding
        self.results: Dict[int, Dict[str, np.ndarray]] = {}
        self.dev = torch.device("cuda", torch.cuda.current_device())
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget_bytes = int(0.8 * free)
        self.budget = int(hbm_budget_bytes)
        self.row_b = row_bytes(k)
        # resident maps (map id -> target), counted before anything else
        self.setup_ctx = lkc.Context()
        self.maps: Dict[int, object] = {}
        self._next_id = 0
        for p in targets_points:
            self.add_map(p, _init=True)
        avail = self.budget - self.resident_bytes
        per_q = n_slots * SCRATCH_BYTES_PER_QUERY + self.row_b
        cap = min(max_rows, avail // per_q)
        if cap < 1:
            raise ValueError("HBM budget too small for one query beside the resident maps")
        self.capacity = int(cap)
        self.fixed_bytes = n_slots * SCRATCH_BYTES_PER_QUERY * self.capacity
        self.pool: Dict[int, List[_BufferSet]] = collections.defaultdict(list)
        self.set_bytes = 0            # bytes of every buffer set (idle or in flight)
        self.inflight_bytes = 0
        self.slots = []
        for _ in range(n_slots):
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                ctx = lkc.Context()
                ctx.reserve(self.capacity)
            q_host = torch.empty((self.capacity, 3), dtype=torch.float32, pin_memory=True)
            self.slots.append(dict(stream=st, ctx=ctx, tset=None, q_host=q_host,
                                   done=torch.cuda.Event(), bufs=None, n=0, offsets=None))
        self._rebuild_sets()

    # ---- maps ----------------------------------------------------------
    @property
    def resident_bytes(self) -> int:
        return int(sum(t.info()["device_bytes"] for t in self.maps.values()))

    def add_map(self, points: np.ndarray, _init: bool = False) -> int:
        """Build a resident map; returns its id.  Refused (ValueError) when
        its bytes do not fit the budget beside what is already held."""
        torch = self.torch
        if not _init:
            self._require_idle()
        p = torch.from_numpy(np.ascontiguousarray(points, np.float32)).to(self.dev)
        t = self.lkc.lkc_build_target(self.setup_ctx, p, self.cell)
        torch.cuda.synchronize()
        del p                      # the target holds its own copy
        mid = self._next_id
        self._next_id += 1
        self.maps[mid] = t
        if not _init:
            used = self.resident_bytes + self.fixed_bytes
            if used + self.set_bytes > self.budget:
                self._evict(used + self.set_bytes - self.budget)
            if used + self.set_bytes > self.budget:
                del self.maps[mid]
                t.free()
                raise ValueError("map does not fit the HBM budget")
            self._rebuild_sets()
        return mid

    def remove_map(self, map_id: int) -> None:
        self._require_idle()
        t = self.maps.pop(map_id)
        t.free()
        self._rebuild_sets()

    def has_map(self, map_id: int) -> bool:
        return map_id in self.maps

    def _require_idle(self):
        if any(s["bufs"] is not None for s in getattr(self, "slots", [])):
            raise RuntimeError("maps change only while no batch is in flight")

    def _rebuild_sets(self):
        """Target-set tables over the current maps (graphs captured on the
        old tables are dropped)."""
        self.order = sorted(self.maps)
        self.index_of = {m: i for i, m in enumerate(self.order)}
        for bs in self.pool.values():
            for b in bs:
                b.graphs.clear()
        for s in self.slots:
            if s["tset"] is not None:
                s["tset"].free()
                s["tset"] = None
            if self.order:
                with self.torch.cuda.stream(s["stream"]):
                    s["tset"] = self.lkc.TargetSet(s["ctx"], [self.maps[m] for m in self.order],
                                                   self.max_scans)

    # ---- memory --------------------------------------------------------
    def _rows(self, n: int) -> int:
        return min(bucket_rows(n), self.capacity) if self.use_graphs else n

    def max_request_queries(self) -> int:
        free = self.budget - self.resident_bytes - self.fixed_bytes
        n = min(self.capacity, free // self.row_b)
        while n > 0 and self._rows(n) * self.row_b > free:
            n -= max(1, n // 64)
        return max(0, int(n))

    def _evict(self, need: int) -> None:
        """Free idle buffer sets (largest first) until `need` bytes are freed."""
        for rows in sorted(self.pool, reverse=True):
            while self.pool[rows] and need > 0:
                self.pool[rows].pop()
                self.set_bytes -= rows * self.row_b
                need -= rows * self.row_b

    def reserve(self, slot: int, batch: List[ServeRequest]) -> bool:
        n = sum(r.points.shape[0] for r in batch)
        rows = self._rows(n)
        if self.pool.get(rows):
            b = self.pool[rows].pop()
        else:
            free = self.budget - self.resident_bytes - self.fixed_bytes - self.set_bytes
            need = rows * self.row_b
            if need > free:
                self._evict(need - free)
                free = self.budget - self.resident_bytes - self.fixed_bytes - self.set_bytes
                if need > free:
                    return False
            b = _BufferSet(self.torch, self.dev, rows, self.k)
            self.set_bytes += need
        self.slots[slot]["bufs"] = b
        self.inflight_bytes += rows * self.row_b
        return True

    def memory(self) -> Dict[str, int]:
        return {"budget": self.budget, "resident": self.resident_bytes,
                "fixed": self.fixed_bytes, "sets": self.set_bytes,
                "inflight": self.inflight_bytes}

    # ---- batches -------------------------------------------------------
    def _call(self, s, b: _BufferSet):
        self.lkc.lkc_knn_cov_batched(s["ctx"], s["tset"], b.q_dev, self.k, self.radius,
                                     self.eps, out=b.out, cfg=self.cfg)

    def launch(self, slot: int, batch: List[ServeRequest]) -> None:
        torch = self.torch
        s = self.slots[slot]
        b = s["bufs"]
        sizes = [r.points.shape[0] for r in batch]
        n = int(sum(sizes))
        total = b.rows
        qh = s["q_host"].numpy()
        off = 0
        scans = []
        for r, m in zip(batch, sizes):
            qh[off:off + m] = r.points
            scans.append((off, m, self.index_of[r.map_id]))
            off += m
        if total > n:
            scans.append((n, total - n, 0))
        with torch.cuda.stream(s["stream"]):
            b.q_dev[:n].copy_(s["q_host"][:n], non_blocking=True)
            if total > n:
                b.q_dev[n:total].fill_(float("nan"))
            s["tset"].stage(scans)
            g = b.graphs.get(slot) if self.use_graphs else None
            if g is None and self.use_graphs and self.capture_new:
                self._call(s, b)              # warm-up outside the capture
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=s["stream"]):
                    self._call(s, b)
                b.graphs[slot] = g
            if g is not None:
                g.replay()
            else:
                self._call(s, b)
            s["done"].record(s["stream"])
        s["n"] = n
        s["offsets"] = np.cumsum([0] + sizes)

    def warm(self, sizes: Iterable[int]) -> int:
        """Allocate the buffer sets of the buckets of `sizes` and capture
        their graphs on every slot ahead of a stream (zero queries against
        the first map); returns the number of buckets.  Set capture_new to
        False afterwards to keep captures out of the stream."""
        buckets = sorted({self._rows(int(n)) for n in sizes if 0 < int(n) <= self.capacity})
        if not self.order:
            return 0
        for rows in buckets:
            for slot in range(self.n_slots):
                req = ServeRequest(-1, 0.0, self.order[0], np.zeros((rows, 3), np.float32))
                if not self.reserve(slot, [req]):
                    return buckets.index(rows)
                self.launch(slot, [req])
                self.slots[slot]["done"].synchronize()
                keep, self.keep_results = self.keep_results, False
                self.finish(slot, [req])
                self.keep_results = keep
        return len(buckets)

    def poll(self, slot: int) -> bool:
        return self.slots[slot]["done"].query()

    def finish(self, slot: int, batch: List[ServeRequest]) -> None:
        s = self.slots[slot]
        b = s["bufs"]
        if self.keep_results:
            offs = s["offsets"]
            host = {key: v[:s["n"]].cpu().numpy() for key, v in b.out.items()}
            for i, r in enumerate(batch):
                self.results[r.rid] = {key: v[offs[i]:offs[i + 1]].copy()
                                       for key, v in host.items()}
        s["bufs"] = None
        self.inflight_bytes -= b.rows * self.row_b
        self.pool[b.rows].append(b)

    def target(self, map_id: int):
        return self.maps[map_id]

    def close(self):
        self.torch.cuda.synchronize()
        self.pool.clear()
        for s in self.slots:
            if s["tset"] is not None:
                s["tset"].free()
            s["ctx"].close()
        for t in self.maps.values():
            t.free()
        self.maps.clear()
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
        lkc.lkc_knn_cov(ctx, ex.target(r.map_id), q, ex.k, ex.radius, ex.eps, cfg=ex.cfg)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - rel)
    wall = time.perf_counter() - t0
    ctx.close()
    n = len(reqs)
    return {"latency_s": np.array(lat), "wall_s": wall,
            "queries": int(sum(r.points.shape[0] for r in reqs)), "requests": n,
            "completed": n, "status_counts": {DONE: n, UNKNOWN_MAP: 0, OVER_BUDGET: 0,
                                              CANCELLED: 0},
            "deferred": 0, "batches": n, "mean_batch_requests": 1.0}
