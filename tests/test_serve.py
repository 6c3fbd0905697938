"""Scheduler of the request loop, on the CPU with a modelled executor.

The executor models a batch as taking `a + b * queries` seconds of device
time on its slot; the clock is simulated (it advances only when the loop
idles), so the tests are deterministic.
"""
import collections
import math

import numpy as np
import pytest

from paper_2308_07173_amd import serve, workloads


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def idle(self, dt=1e-5):
        self.t += dt


class ModelExecutor(serve.Executor):
    """Batch time a + b * queries on its slot; device bytes modelled as
    `row` bytes per query against `budget`, beside resident maps of given
    sizes (map id -> bytes)."""

    def __init__(self, clock, n_slots=2, capacity=300_000, a=2e-4, b=2e-9, budget=math.inf,
                 maps=None, row=100):
        self.clock, self.n_slots, self.capacity, self.a, self.b = clock, n_slots, capacity, a, b
        self.budget, self.row = budget, row
        self.maps = dict({0: 0, 1: 0, 2: 0, 3: 0} if maps is None else maps)
        self.busy_until = [None] * n_slots
        self.claimed = [0] * n_slots
        self.launched = []
        self.max_inflight = 0
        self.max_claimed = 0

    def has_map(self, map_id):
        return map_id in self.maps

    def resident(self):
        return sum(self.maps.values())

    def max_request_queries(self):
        free = self.budget - self.resident()
        return self.capacity if math.isinf(free) else min(self.capacity, int(free // self.row))

    def reserve(self, slot, batch):
        need = self.row * sum(r.points.shape[0] for r in batch)
        if self.resident() + sum(self.claimed) + need > self.budget:
            return False
        self.claimed[slot] = need
        self.max_claimed = max(self.max_claimed, sum(self.claimed))
        return True

    def launch(self, slot, batch):
        n = sum(r.points.shape[0] for r in batch)
        assert n <= self.capacity
        assert self.claimed[slot] == self.row * n          # reserved first
        self.busy_until[slot] = self.clock() + self.a + self.b * n
        self.launched.append((self.clock(), slot, [r.rid for r in batch]))
        self.max_inflight = max(self.max_inflight, sum(x is not None for x in self.busy_until))

    def poll(self, slot):
        return self.busy_until[slot] is not None and self.clock() >= self.busy_until[slot]

    def finish(self, slot, batch):
        self.busy_until[slot] = None
        self.claimed[slot] = 0

    def memory(self):
        return {"inflight": sum(self.claimed)}


def make_requests(n=60, seed=0, rate=60.0, nmin=1000, nmax=100_000, n_maps=4):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        m = int(rng.integers(nmin, nmax + 1))
        out.append(serve.ServeRequest(i, t, int(rng.integers(0, n_maps)),
                                      np.zeros((m, 3), np.float32)))
    return out


def test_plan_batch_is_fifo_and_respects_capacity():
    reqs = [serve.ServeRequest(i, 0.0, 0, np.zeros((n, 3), np.float32))
            for i, n in enumerate([40, 30, 50, 10])]
    q = collections.deque(reqs)
    b = serve.plan_batch(q, 100)
    assert [r.rid for r in b] == [0, 1]          # request 2 does not fit; 3 must not overtake
    assert [r.rid for r in q] == [2, 3]
    assert serve.plan_batch(collections.deque(), 100) == []


def test_serve_loop_completes_everything_with_continuous_batching():
    clock = SimClock()
    ex = ModelExecutor(clock)
    reqs = make_requests()
    res = serve.serve_loop(reqs, ex, time_scale=1.0, clock=clock, idle=clock.idle)
    assert res["requests"] == len(reqs) and len(res["latency_s"]) == len(reqs)
    assert np.all(res["latency_s"] > 0)
    seen = [rid for _, _, ids in ex.launched for rid in ids]
    assert sorted(seen) == list(range(len(reqs)))   # every request exactly once
    assert seen == sorted(seen)                      # FIFO across batches
    assert ex.max_inflight == 2                      # both slots used at once
    # a request is never launched before it arrived
    arrival = {r.rid: r.t_arrival for r in reqs}
    for t, _, ids in ex.launched:
        assert all(arrival[i] <= t + 1e-12 for i in ids)


def test_open_loop_batches_fill_capacity():
    clock = SimClock()
    ex = ModelExecutor(clock, capacity=250_000)
    reqs = make_requests(n=40, seed=3)
    res = serve.serve_loop(reqs, ex, time_scale=math.inf, clock=clock, idle=clock.idle)
    assert res["batches"] < len(reqs)                # requests were batched together
    for _, _, ids in ex.launched:
        assert sum(reqs[i].points.shape[0] for i in ids) <= 250_000


def test_small_budget_still_serves_all_and_queues():
    clock = SimClock()
    ex = ModelExecutor(clock, n_slots=2, capacity=100_000)
    reqs = make_requests(n=30, seed=5, rate=1000.0, nmax=100_000)
    res = serve.serve_loop(reqs, ex, time_scale=1.0, clock=clock, idle=clock.idle)
    assert res["requests"] == 30
    # under overload, later requests wait: latency grows along the stream
    lat = res["latency_s"]
    assert lat[-5:].mean() > lat[:5].mean()


def test_oversized_request_is_refused_and_the_rest_served():
    clock = SimClock()
    ex = ModelExecutor(clock, capacity=1000)
    reqs = [serve.ServeRequest(0, 0.0, 0, np.zeros((500, 3), np.float32)),
            serve.ServeRequest(1, 0.0, 0, np.zeros((1001, 3), np.float32)),
            serve.ServeRequest(2, 0.0, 0, np.zeros((600, 3), np.float32))]
    res = serve.serve_loop(reqs, ex, clock=clock, idle=clock.idle)
    assert res["status"] == {0: serve.DONE, 1: serve.OVER_BUDGET, 2: serve.DONE}
    assert res["completed"] == 2 and len(res["latency_s"]) == 2


def test_unknown_map_is_rejected_per_request():
    clock = SimClock()
    ex = ModelExecutor(clock, maps={0: 0, 2: 0})
    reqs = make_requests(n=40, seed=11, n_maps=4)
    res = serve.serve_loop(reqs, ex, time_scale=1.0, clock=clock, idle=clock.idle)
    for r in reqs:
        want = serve.DONE if r.map_id in (0, 2) else serve.UNKNOWN_MAP
        assert res["status"][r.rid] == want
    launched = {rid for _, _, ids in ex.launched for rid in ids}
    assert launched == {r.rid for r in reqs if r.map_id in (0, 2)}
    assert res["status_counts"][serve.UNKNOWN_MAP] == sum(r.map_id in (1, 3) for r in reqs) > 0


def test_over_budget_batch_is_deferred_then_admitted():
    """Two slots, but the budget holds one 60k-query request at a time
    beside the resident maps: the second waits for the first to finish,
    then runs; the claimed bytes never exceed the budget."""
    clock = SimClock()
    maps = {0: 2_000_000, 1: 3_000_000}
    ex = ModelExecutor(clock, capacity=100_000, budget=5_000_000 + 100 * 80_000, maps=maps)
    reqs = [serve.ServeRequest(i, 0.0, i % 2, np.zeros((60_000, 3), np.float32))
            for i in range(4)]
    res = serve.serve_loop(reqs, ex, time_scale=math.inf, clock=clock, idle=clock.idle)
    assert all(v == serve.DONE for v in res["status"].values())
    assert res["deferred"] >= 3
    assert ex.max_inflight == 1                       # never two batches at once
    assert ex.max_claimed <= ex.budget - ex.resident()
    assert [ids for _, _, ids in ex.launched] == [[0], [1], [2], [3]]


def test_request_that_never_fits_is_refused_while_others_run():
    clock = SimClock()
    ex = ModelExecutor(clock, capacity=100_000, budget=100 * 50_000, maps={0: 0})
    sizes = [10_000, 70_000, 20_000, 49_000]
    reqs = [serve.ServeRequest(i, 0.001 * i, 0, np.zeros((n, 3), np.float32))
            for i, n in enumerate(sizes)]
    res = serve.serve_loop(reqs, ex, time_scale=1.0, clock=clock, idle=clock.idle)
    assert res["status"] == {0: serve.DONE, 1: serve.OVER_BUDGET, 2: serve.DONE,
                             3: serve.DONE}


def test_resident_maps_count_against_the_budget():
    """Loading a larger map leaves less for requests: one that fit before
    is refused afterwards, and the next stream still serves the rest."""
    clock = SimClock()
    ex = ModelExecutor(clock, capacity=100_000, budget=10_000_000, maps={0: 1_000_000})
    big = lambda rid: serve.ServeRequest(rid, 0.0, 0, np.zeros((80_000, 3), np.float32))
    small = lambda rid: serve.ServeRequest(rid, 0.0, 0, np.zeros((5_000, 3), np.float32))
    res = serve.serve_loop([big(0), small(1)], ex, clock=clock, idle=clock.idle)
    assert res["status"] == {0: serve.DONE, 1: serve.DONE}
    ex.maps[1] = 4_000_000                            # a second resident map
    res = serve.serve_loop([big(2), small(3)], ex, clock=clock, idle=clock.idle)
    assert res["status"] == {2: serve.OVER_BUDGET, 3: serve.DONE}


def test_cancel_while_queued():
    """Overloaded stream: requests cancelled while queued are never
    launched; a cancel after launch lets the request complete; a cancel of
    a request that has not arrived yet drops it on arrival."""
    clock = SimClock()
    ex = ModelExecutor(clock, n_slots=1, capacity=50_000, a=5e-3)
    reqs = [serve.ServeRequest(i, 0.001 * i, 0, np.zeros((40_000, 3), np.float32))
            for i in range(10)]
    # at 2.5 ms request 0 runs and 1, 2 are queued; 9 arrives at 9 ms; at
    # 12 ms request 6 (arrived at 6 ms) is still queued behind 3, 4, 5
    cancels = [(0.0025, 0), (0.0025, 2), (0.0025, 9), (0.012, 6)]
    res = serve.serve_loop(reqs, ex, time_scale=1.0, clock=clock, idle=clock.idle,
                           cancels=cancels)
    st = res["status"]
    launched = {rid for _, _, ids in ex.launched for rid in ids}
    assert st[0] == serve.DONE and res["late_cancels"] == 1     # already running
    for rid in (2, 6, 9):
        assert st[rid] == serve.CANCELLED and rid not in launched
    assert all(st[i] == serve.DONE for i in (1, 3, 4, 5, 7, 8))
    assert res["completed"] == 7
    # FIFO among the rest
    order = [rid for _, _, ids in ex.launched for rid in ids]
    assert order == [0, 1, 3, 4, 5, 7, 8]


def test_open_loop_cancel_drops_queued_requests():
    clock = SimClock()
    ex = ModelExecutor(clock, n_slots=1, capacity=50_000)
    reqs = [serve.ServeRequest(i, 0.0, 0, np.zeros((30_000, 3), np.float32)) for i in range(5)]
    res = serve.serve_loop(reqs, ex, time_scale=math.inf, clock=clock, idle=clock.idle,
                           cancels=[(0.0, 1), (0.0, 3)])
    assert [res["status"][i] for i in range(5)] == [serve.DONE, serve.CANCELLED, serve.DONE,
                                                   serve.CANCELLED, serve.DONE]
    assert [ids for _, _, ids in ex.launched] == [[0], [2], [4]]


def test_bucket_rows_pad_at_most_an_eighth():
    for n in list(range(1, 5000, 37)) + [131_072, 131_073, 1_000_000, 3_757_703]:
        b = serve.bucket_rows(n)
        assert b >= n and b >= 1024
        if n > 1024:
            assert b <= n * 1.125 + 1
    assert serve.bucket_rows(1 << 20) == 1 << 20


def test_bytes_per_query_accounts_outputs():
    # query + idx/d2 rows + count + mean + cov + reg + valid, + search scratch
    assert serve.row_bytes(20) == 12 + 160 + 4 + 12 + 36 + 36 + 1
    assert serve.bytes_per_query(20) == serve.row_bytes(20) + serve.SCRATCH_BYTES_PER_QUERY


def test_served_schedule_shape():
    reqs = workloads.served_schedule(duration=10.0, seed=5)
    # three sensors at 20 Hz for 10 s: about 600 requests
    assert 450 < len(reqs) < 750
    ts = [r.t_arrival for r in reqs]
    assert ts == sorted(ts)
    assert all(10_000 <= r.n_points <= 131_072 for r in reqs)
    assert {r.map_id for r in reqs} == {0, 1, 2, 3}
