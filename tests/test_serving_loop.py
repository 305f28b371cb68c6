"""CPU tests of the serving request loop (arrival replay, completion accounting, percentiles)
with a scripted stand-in for the GPU server, and of the seeded serving workload generator."""
import math

import pytest

import cmcg_inputs as ci
from paper_1903_12522_amd import serving


class ScriptedServer:
    """Completes each request a fixed number of steps after admission; admits at most `slots`."""

    def __init__(self, slots=2, work=3):
        self.slots, self.work = slots, work
        self.queue, self.running, self.done = [], {}, set()
        self.next = 1
        self.max_running = 0

    def submit(self, problem, precision="fp32", tol=1e-6, max_iter=1000):
        rid = self.next
        self.next += 1
        self.queue.append(rid)
        return rid

    def step(self):
        while self.queue and len(self.running) < self.slots:
            self.running[self.queue.pop(0)] = self.work
        for rid in list(self.running):
            self.running[rid] -= 1
            if self.running[rid] == 0:
                del self.running[rid]
                self.done.add(rid)
        self.max_running = max(self.max_running, len(self.running))
        return len(self.running), len(self.queue)

    def poll(self, rid):
        if rid in self.done:
            return 2, None, {"iterations": 7, "steps_per_period": 16, "rel_residual": 1e-7,
                             "grid_updates": 1e6}, 0
        return (1 if rid in self.running else 0), None, None, 0


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.01          # every clock read advances 10 ms
        return self.t

    def sleep(self, d):
        self.t += d


def test_loop_completes_all_and_respects_slots():
    reqs = ci.serving_requests(count=12, rate_hz=20.0, seed=3, build_fields=False)
    srv = ScriptedServer(slots=2, work=3)
    clk = FakeClock()
    recs, summ = serving.run(srv, reqs, clock=clk, sleep=clk.sleep)
    assert summ["requests"] == 12 and summ["completed"] == 12 and summ["converged"] == 12
    assert srv.max_running <= 2
    assert sorted(r.index for r in recs) == list(range(12))
    for r in recs:
        assert r.latency_s > 0 and r.done_s >= r.arrival_s
    assert summ["p50_latency_s"] <= summ["p99_latency_s"] <= summ["max_latency_s"]


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert serving.percentile(xs, 50) == 50
    assert serving.percentile(xs, 99) == 99
    assert serving.percentile([3.0], 99) == 3.0


def test_serving_workload_is_seeded_and_in_range():
    a = ci.serving_requests(count=64, seed=11, build_fields=False)
    b = ci.serving_requests(count=64, seed=11, build_fields=False)
    assert [r.arrival_s for r in a] == [r.arrival_s for r in b]
    assert all(x.arrival_s <= y.arrival_s for x, y in zip(a, a[1:]))
    assert a[0].arrival_s == 0.0
    sides = {r.problem.n[0] for r in a}
    assert sides <= {256, 512, 1024, 2048} and len(sides) >= 3
    for r in a:
        W = r.problem.omega / (2 * math.pi)
        assert 4.0 <= W <= 64.0
    # mean inter-arrival close to 1 / 20 s
    gaps = [y.arrival_s - x.arrival_s for x, y in zip(a, a[1:])]
    assert 0.03 < sum(gaps) / len(gaps) < 0.08
