"""Scheduling logic of the continuous-batching server, on a fake backend and clock."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2607_25161_amd.serving import BatchEngine, Request, poisson_arrivals


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt):
        self.t += dt


class FakeSusp:
    def __init__(self, n_bead):
        self.n_bead = n_bead


class FakeBackend:
    """Memory = 1000 bytes per bead; a step costs 1 us per active bead on the fake clock."""

    def __init__(self, clock, budget, slots, fail=()):
        self.clock, self.budget, self.slots = clock, budget, slots
        self.active = {}
        self.fail = set(fail)
        self.peak_bytes = 0
        self.peak_slots = 0
        self.steps = {}

    def estimate(self, req):
        return 1000 * req.suspension.n_bead

    def used_bytes(self):
        return sum(1000 * r.suspension.n_bead for r in self.active.values())

    def free_device_bytes(self):
        return self.budget - self.used_bytes()

    def admit(self, req):
        if len(self.active) >= self.slots or self.used_bytes() + self.estimate(req) > self.budget:
            return None
        slot = min(set(range(self.slots)) - set(self.active))
        self.active[slot] = req
        self.peak_bytes = max(self.peak_bytes, self.used_bytes())
        self.peak_slots = max(self.peak_slots, len(self.active))
        return slot

    def step(self, dt, counts=None):
        counts = counts or {slot: 1 for slot in self.active}
        # the systems work side by side: a tick lasts as long as its busiest system
        self.clock.advance(1e-6 * max(r.suspension.n_bead * counts[slot] for slot, r in self.active.items()))
        out = {}
        for slot, r in self.active.items():
            out[slot] = 0
            for _ in range(counts[slot]):
                self.steps[r.rid] = self.steps.get(r.rid, 0) + 1
                if r.rid in self.fail and self.steps[r.rid] == 2:
                    out[slot] = -3
                    break
        return out

    def retire(self, slot):
        r = self.active.pop(slot)
        return ("state", r.rid)


def _requests(sizes, arrivals, n_steps=5):
    return [Request(rid=k, suspension=FakeSusp(n), n_steps=n_steps, arrival=float(t))
            for k, (n, t) in enumerate(zip(sizes, arrivals))]


def test_every_request_runs_its_steps_and_resources_hold():
    clk = FakeClock()
    be = FakeBackend(clk, budget=10_000_000, slots=4)
    eng = BatchEngine(be, max_slots=4, clock=clk)
    rng = np.random.default_rng(0)
    sizes = rng.integers(100, 5000, size=40)
    rep = eng.run(_requests(sizes, poisson_arrivals(rng, 40, rate=200.0), n_steps=7))
    assert rep["completed"] == 40 and rep["failed"] == 0
    assert all(be.steps[k] == 7 for k in range(40))
    assert be.peak_slots <= 4 and be.peak_bytes <= 10_000_000
    assert rep["bead_steps"] == 7 * int(sizes.sum())
    assert all(r.result == ("state", r.rid) for r in eng.done)


def test_continuous_batching_refills_freed_slot_at_next_step():
    clk = FakeClock()
    be = FakeBackend(clk, budget=1 << 40, slots=2)
    eng = BatchEngine(be, max_slots=2, clock=clk)
    reqs = [Request(0, FakeSusp(100), 2), Request(1, FakeSusp(100), 10), Request(2, FakeSusp(100), 3)]
    # equal sizes: one step per tick each
    for r in reqs:
        eng.submit(r)
    eng.tick()                       # admits 0 and 1
    assert set(r.rid for r in eng.active.values()) == {0, 1}
    eng.tick()                       # request 0 finishes its 2 steps
    assert reqs[0].finished is not None and len(eng.active) == 1
    eng.tick()                       # request 2 joins without waiting for request 1
    assert set(r.rid for r in eng.active.values()) == {1, 2}
    assert reqs[2].steps_done == 1 and reqs[1].steps_done == 3


def test_admission_by_memory_is_first_come_first_served():
    clk = FakeClock()
    be = FakeBackend(clk, budget=3_000_000, slots=8)
    eng = BatchEngine(be, max_slots=8, clock=clk)
    reqs = [Request(0, FakeSusp(2000), 3), Request(1, FakeSusp(2000), 3), Request(2, FakeSusp(500), 3)]
    for r in reqs:
        eng.submit(r)
    eng.tick()
    # request 1 does not fit next to request 0; request 2 would, but may not overtake
    assert [r.rid for r in eng.active.values()] == [0]
    while eng.active or eng.queue:
        eng.tick()
        assert be.used_bytes() <= 3_000_000
    assert [r.rid for r in sorted(eng.done, key=lambda r: (r.started, r.rid))] == [0, 1, 2]


def test_oversized_request_is_rejected_not_blocking():
    clk = FakeClock()
    be = FakeBackend(clk, budget=1_000_000, slots=2)
    eng = BatchEngine(be, max_slots=2, clock=clk)
    rep = eng.run(_requests([5000, 300, 200], [0.0, 0.0, 0.0], n_steps=2))
    assert rep["completed"] == 2 and rep["failed"] == 1
    bad = [r for r in eng.done if r.status != 0]
    assert bad[0].rid == 0 and bad[0].status == -7


def test_failed_solve_retires_only_that_request():
    clk = FakeClock()
    be = FakeBackend(clk, budget=1 << 40, slots=4, fail={1})
    eng = BatchEngine(be, max_slots=4, clock=clk)
    rep = eng.run(_requests([100, 200, 300], [0.0, 0.0, 0.0], n_steps=4))
    assert rep["failed"] == 1 and rep["completed"] == 2
    r1 = [r for r in eng.done if r.rid == 1][0]
    assert r1.status == -3 and r1.steps_done == 1
    assert be.steps[0] == 4 and be.steps[2] == 4


def test_latency_accounting_on_fake_clock():
    clk = FakeClock()
    be = FakeBackend(clk, budget=1 << 40, slots=1)
    eng = BatchEngine(be, max_slots=1, clock=clk)
    # one slot: requests run back to back; each step of 1000 beads costs 1 ms
    rep = eng.run(_requests([1000] * 4, [0.0, 0.0, 0.0, 0.0], n_steps=5))
    lat = sorted(r.latency for r in eng.done)
    assert lat == pytest.approx([5e-3, 10e-3, 15e-3, 20e-3])
    assert rep["p50_latency_s"] == pytest.approx(np.percentile(lat, 50))
    assert rep["p99_latency_s"] == pytest.approx(np.percentile(lat, 99))
    assert rep["span_s"] == pytest.approx(20e-3)
    assert rep["bead_solves_per_s"] == pytest.approx(4 * 5 * 1000 / 20e-3)


def test_idle_engine_waits_for_arrivals():
    clk = FakeClock()
    be = FakeBackend(clk, budget=1 << 40, slots=2)
    eng = BatchEngine(be, max_slots=2, clock=clk)
    rep = eng.run(_requests([1000, 1000], [0.0, 1.0], n_steps=1))
    r0, r1 = sorted(eng.done, key=lambda r: r.rid)
    assert r0.latency == pytest.approx(1e-3) and r1.latency == pytest.approx(1e-3)
    assert r1.started >= r1.arrival
    assert rep["span_s"] == pytest.approx(1.001)


def test_poisson_arrivals_rate():
    rng = np.random.default_rng(1)
    t = poisson_arrivals(rng, 20000, rate=4.0)
    assert np.all(np.diff(t) > 0)
    assert t[-1] / 20000 == pytest.approx(0.25, rel=0.03)


class UnderEstimatingBackend(FakeBackend):
    """The estimate says a request fits, but the batch refuses it even when empty (a held
    size above the estimate): the engine must reject it instead of retrying forever."""

    def estimate(self, req):
        return 1

    def admit(self, req):
        if req.suspension.n_bead > 4000:
            return None
        return super().admit(req)


def test_request_refused_by_an_empty_batch_is_rejected():
    clk = FakeClock()
    be = UnderEstimatingBackend(clk, budget=1 << 40, slots=2)
    eng = BatchEngine(be, max_slots=2, clock=clk)
    rep = eng.run(_requests([5000, 300], [0.0, 0.0], n_steps=2))
    assert rep["completed"] == 1 and rep["failed"] == 1
    bad = [r for r in eng.done if r.status != 0]
    assert bad[0].rid == 0 and bad[0].status == -7


def test_small_requests_take_several_steps_per_tick():
    """A request 4 times smaller than the largest active one takes 4 steps per tick (capped
    by its remaining steps), so it finishes in a quarter of the ticks."""
    clk = FakeClock()
    be = FakeBackend(clk, budget=1 << 40, slots=2)
    eng = BatchEngine(be, max_slots=2, clock=clk, max_steps_per_tick=8)
    big, small = Request(0, FakeSusp(4000), 8), Request(1, FakeSusp(1000), 8)
    eng.submit(big)
    eng.submit(small)
    eng.tick()
    assert small.steps_done == 4 and big.steps_done == 1
    eng.tick()
    assert small.finished is not None and small.steps_done == 8 and big.steps_done == 2
    while eng.active:
        eng.tick()
    assert be.steps[0] == 8 and be.steps[1] == 8
    # the small request's latency is two ticks of the big one
    assert small.latency == pytest.approx(2 * 4000e-6)


def test_one_step_per_tick_when_multi_step_is_off():
    clk = FakeClock()
    be = FakeBackend(clk, budget=1 << 40, slots=2)
    eng = BatchEngine(be, max_slots=2, clock=clk, max_steps_per_tick=1)
    eng.submit(Request(0, FakeSusp(4000), 3))
    eng.submit(Request(1, FakeSusp(1000), 3))
    eng.tick()
    assert [r.steps_done for r in eng.active.values()] == [1, 1]
