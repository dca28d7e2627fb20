"""Scheduler of the serving loop on the CPU, against a fake executor on a
virtual clock: slot and budget limits, FIFO admission, continuous joining of
late arrivals, completion of every request, latency statistics."""
import math

import numpy as np
import pytest

from paper_1807_11830_amd.serving import Request, Scheduler, make_requests, stats


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-9)


class FakeExecutor:
    """Slots and a byte budget; every admitted request needs `iters` steps;
    one step costs step_cost seconds of virtual time."""

    def __init__(self, clock, slots=4, budget=10_000, step_cost=1e-3):
        self.clock, self.slots, self.budget, self.step_cost = clock, slots, budget, step_cost
        self.live = {}
        self.used = 0
        self.admit_order = []
        self.max_live = 0
        self.max_used = 0
        self.done = []

    def fp(self, r):
        return r.n * r.n // 64

    def admit(self, r):
        if len(self.live) >= self.slots or self.used + self.fp(r) > self.budget:
            return False
        self.live[r.id] = [r, 0]
        self.used += self.fp(r)
        self.admit_order.append(r.id)
        self.max_live = max(self.max_live, len(self.live))
        self.max_used = max(self.max_used, self.used)
        return True

    def step(self):
        self.clock.t += self.step_cost
        for v in self.live.values():
            v[1] += 1

    def poll(self):
        out = [rid for rid, (r, k) in self.live.items() if k >= r.iters]
        for rid in out:
            r, _ = self.live.pop(rid)
            self.used -= self.fp(r)
            self.done.append(rid)
        return out

    def release(self, r):
        r.result = "ok"


def test_all_finish_within_limits():
    clk = VClock()
    ex = FakeExecutor(clk, slots=5, budget=5000)
    reqs = make_requests(200, rate=400.0, iters=7)
    st = Scheduler(ex, clock=clk, sleep=clk.sleep).run(reqs)
    assert st.n == 200 and all(r.result == "ok" for r in reqs)
    assert ex.max_live <= 5 and ex.max_used <= 5000
    assert all(r.finished >= r.admitted >= r.arrival - 1e-12 for r in reqs)
    # FIFO: admission follows arrival order
    order = [r.id for r in sorted(reqs, key=lambda r: (r.arrival, r.id))]
    assert ex.admit_order == order


def test_late_arrivals_join_running_batch():
    clk = VClock()
    ex = FakeExecutor(clk, slots=8, budget=10**9, step_cost=1e-3)
    reqs = [Request(0, 0.0, 128, 8, 2, 20), Request(1, 0.005, 128, 8, 2, 20),
            Request(2, 0.010, 192, 16, 3, 20)]
    Scheduler(ex, clock=clk, sleep=clk.sleep).run(reqs)
    # request 1 and 2 were admitted while request 0 was still running
    assert reqs[1].admitted < reqs[0].finished and reqs[2].admitted < reqs[0].finished
    assert ex.max_live == 3


def test_budget_blocks_then_admits():
    clk = VClock()
    ex = FakeExecutor(clk, slots=10, budget=1024)  # fits one 256x256 request at a time
    reqs = [Request(i, 0.0, 256, 8, 2, 5) for i in range(3)]
    Scheduler(ex, clock=clk, sleep=clk.sleep).run(reqs)
    assert ex.max_live == 1
    assert reqs[0].finished <= reqs[1].admitted <= reqs[1].finished <= reqs[2].admitted


def test_oversized_request_raises():
    clk = VClock()
    ex = FakeExecutor(clk, slots=2, budget=10)
    with pytest.raises(RuntimeError, match="never be admitted"):
        Scheduler(ex, clock=clk, sleep=clk.sleep).run([Request(0, 0.0, 320, 8, 2, 5)])


def test_stats():
    reqs = [Request(i, float(i), 128, 8, 2, 1) for i in range(100)]
    for r in reqs:
        r.finished = r.arrival + (r.id + 1) * 1e-3
    s = stats(reqs)
    lat = np.array([(i + 1) * 1e-3 for i in range(100)])
    assert math.isclose(s.p50, np.percentile(lat, 50))
    assert math.isclose(s.p99, np.percentile(lat, 99))
    assert math.isclose(s.throughput, 100 / (99 + 0.1))
