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
    def __init__(self, clock, n_slots=2, capacity=300_000, a=2e-4, b=2e-9):
        self.clock, self.n_slots, self.capacity, self.a, self.b = clock, n_slots, capacity, a, b
        self.busy_until = [None] * n_slots
        self.launched = []
        self.max_inflight = 0

    def launch(self, slot, batch):
        n = sum(r.points.shape[0] for r in batch)
        assert n <= self.capacity
        self.busy_until[slot] = self.clock() + self.a + self.b * n
        self.launched.append((self.clock(), slot, [r.rid for r in batch]))
        self.max_inflight = max(self.max_inflight, sum(x is not None for x in self.busy_until))

    def poll(self, slot):
        return self.busy_until[slot] is not None and self.clock() >= self.busy_until[slot]

    def finish(self, slot, batch):
        self.busy_until[slot] = None


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


def test_oversized_request_is_rejected():
    clock = SimClock()
    ex = ModelExecutor(clock, capacity=1000)
    reqs = [serve.ServeRequest(0, 0.0, 0, np.zeros((1001, 3), np.float32))]
    with pytest.raises(ValueError):
        serve.serve_loop(reqs, ex, clock=clock, idle=clock.idle)


def test_bytes_per_query_accounts_outputs():
    # query + idx/d2 rows + count + mean + cov + reg + valid + scratch
    assert serve.bytes_per_query(20) == 12 + 160 + 4 + 12 + 36 + 36 + 1 + 36


def test_served_schedule_shape():
    reqs = workloads.served_schedule(duration=10.0, seed=5)
    # three sensors at 20 Hz for 10 s: about 600 requests
    assert 450 < len(reqs) < 750
    ts = [r.t_arrival for r in reqs]
    assert ts == sorted(ts)
    assert all(10_000 <= r.n_points <= 131_072 for r in reqs)
    assert {r.map_id for r in reqs} == {0, 1, 2, 3}
