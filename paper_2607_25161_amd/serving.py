"""Continuous-batching solve server over the batch C ABI.

Requests are whole simulations (a suspension and a number of time steps).  The
engine admits queued requests while the batch has a free slot and the device
memory estimate of the new system fits the budget and the free device memory;
admitted systems keep their grids, neighbour lists and factors resident; every
engine tick advances every active system by at least one time step (batched
solves + Euler updates).  A tick is paced by its largest system: a system whose
estimated size is k times smaller takes up to k steps in the same tick (at most
max_steps_per_tick), so small requests do not wait on large ones step for step.
Finished requests retire and free their slot and memory, and queued requests
take their place at the next tick.  Latency is measured from a request's arrival
to the end of its last step.

The compute all happens in libfsd (fsd_batch_step); this module only schedules.
The backend and the clock are injectable so the scheduling logic can be tested
without a GPU.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass
import time
from typing import Callable, Deque, Dict, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    suspension: object          # workload with the usual attributes (L, offsets, ...)
    n_steps: int
    arrival: float = 0.0        # seconds on the engine clock
    started: Optional[float] = None
    finished: Optional[float] = None
    steps_done: int = 0
    status: int = 0
    n_bead: int = 0
    result: object = None       # final (com, quat) of the request's aggregates

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class LibBackend:
    """The real backend: one System per request, one fsd_batch for all."""

    def __init__(self, F, mem_budget: int, max_slots: int, params: dict, warm_start: int = 0,
                 lees_edwards: bool = False, drift: int = 0):
        self.F = F
        self.batch = F.Batch(mem_budget, max_slots)
        self.params = params
        self.budget = mem_budget
        self.warm_start = warm_start  # GMRES initial guess of each request's solves (fsd_set_warm_start)
        self.lees_edwards = lees_edwards
        # Brownian drift of requests with kT > 0 (fsd_set_drift: 1 random finite differences,
        # 2 Fixman; 0 none): the drift is what makes the served trajectories sample the
        # equilibrium distribution (Appendix A), at two more solves per step
        self.drift = drift

    def estimate(self, req: Request) -> int:
        """Device bytes the request's system will hold.  On the sheared lattice the library
        grows the grid by sqrt(5)/2 per side; sizing the estimate on a box that much larger
        bounds that grid from above (the other terms only grow with it)."""
        s = req.suspension
        p = self.F.default_params(**self._kw(s))
        L = s.L * (1.25 ** 0.5 if self.lees_edwards else 1.0)
        return self.F.estimate_bytes(p, s.n_bead, s.n_agg, L)

    def _kw(self, s):
        kw = dict(eta=s.eta, radius=s.a, xi=s.xi, ewald_tol=s.ewald_tol, grid=s.grid, r_lub=s.r_lub,
                  r_precond=s.r_precond, gmres_tol=s.gmres_tol, kT=getattr(s, "kT", 0.0))
        kw.update(self.params)
        return kw

    def free_device_bytes(self) -> int:
        try:
            import torch
            free, _ = torch.cuda.mem_get_info()
            return int(free)
        except Exception:
            return 1 << 62

    def admit(self, req: Request):
        s = req.suspension
        sysm = self.F.System.from_suspension(s, lees_edwards=self.lees_edwards, **self.params)
        if self.warm_start:
            sysm.set_warm_start(self.warm_start)
        if self.drift and getattr(s, "kT", 0.0) > 0:
            sysm.set_drift(self.drift)
        slot = self.batch.try_admit(sysm)
        if slot is None:
            sysm.close()
        return slot

    def step(self, dt: float, counts: Optional[Dict[int, int]] = None) -> Dict[int, int]:
        """One tick: counts[slot] time steps per system (one each when None)."""
        if counts is None:
            self.batch.step(dt)
        else:
            self.batch.step_counts(dt, counts)
        return {slot: self.batch.info(slot).status for slot in list(self.batch.systems)}

    def retire(self, slot: int):
        sysm = self.batch.retire(slot)
        state = sysm.state()
        sysm.close()
        return state

    def used_bytes(self) -> int:
        return self.batch.used_bytes()


class BatchEngine:
    def __init__(self, backend, max_slots: int, dt: float = 1e-3, clock: Callable[[], float] = time.perf_counter,
                 mem_budget: Optional[int] = None, max_steps_per_tick: int = 8):
        self.backend = backend
        self.max_slots = max_slots
        self.dt = dt
        self.max_steps_per_tick = max(1, int(max_steps_per_tick))
        self.cost: Dict[int, int] = {}
        self.clock = clock
        self.mem_budget = mem_budget if mem_budget is not None else getattr(backend, "budget", 1 << 62)
        self.queue: Deque[Request] = deque()
        self.active: Dict[int, Request] = {}
        self.done: List[Request] = []
        self.ticks = 0
        self.bead_steps = 0

    def submit(self, req: Request):
        self.queue.append(req)

    def _admit(self):
        # first-come first-served; a request that does not fit waits (no overtaking)
        while self.queue and len(self.active) < self.max_slots:
            req = self.queue[0]
            need = self.backend.estimate(req)
            if need > self.mem_budget:
                self.queue.popleft()
                req.status = -7        # can never fit: rejected
                req.finished = self.clock()
                self.done.append(req)
                continue
            if need > self.backend.free_device_bytes():
                break
            slot = self.backend.admit(req)
            if slot is None:
                if not self.active:
                    # refused by an empty batch: it will never fit
                    self.queue.popleft()
                    req.status = -7
                    req.finished = self.clock()
                    self.done.append(req)
                    continue
                break
            self.queue.popleft()
            req.started = self.clock()
            req.n_bead = req.suspension.n_bead
            self.active[slot] = req
            self.cost[slot] = max(1, need)

    def tick(self):
        """Admit what fits, advance every active request by one step, retire the finished."""
        self._admit()
        if not self.active:
            return False
        # the largest system paces the tick; a system k times smaller takes up to k steps
        ref = max(self.cost[slot] for slot in self.active)
        counts = {slot: max(1, min(self.max_steps_per_tick, ref // self.cost[slot], req.n_steps - req.steps_done))
                  for slot, req in self.active.items()}
        status = self.backend.step(self.dt, counts if self.max_steps_per_tick > 1 else None)
        now = self.clock()
        self.ticks += 1
        for slot, req in list(self.active.items()):
            st = status.get(slot, 0)
            if st != 0:
                req.status = st
            else:
                req.steps_done += counts[slot]
                self.bead_steps += req.n_bead * counts[slot]
            if st != 0 or req.steps_done >= req.n_steps:
                req.finished = now
                req.result = self.backend.retire(slot)
                del self.active[slot]
                del self.cost[slot]
                self.done.append(req)
        return True

    def run(self, requests: List[Request], start: Optional[float] = None, on_tick: Optional[Callable] = None):
        """Open-loop run: requests enter the queue at their arrival times (engine clock).
        on_tick(engine) is called after every engine tick (progress reporting)."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        t0 = self.clock() if start is None else start
        for r in pending:
            r.arrival += t0
        while pending or self.queue or self.active:
            now = self.clock()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            ticked = self.tick()
            if ticked and on_tick is not None:
                on_tick(self)
            if not ticked and pending:
                # idle: wait for the next arrival
                wait = pending[0].arrival - self.clock()
                if wait > 0 and hasattr(self.clock, "advance"):
                    self.clock.advance(wait)
                elif wait > 0:
                    time.sleep(min(wait, 0.05))
        return self.report(t0)

    def report(self, t0: float):
        lat = [r.latency for r in self.done if r.status == 0]
        span = max((r.finished for r in self.done), default=t0) - t0
        fails = {}
        for r in self.done:
            if r.status != 0:
                fails[r.status] = fails.get(r.status, 0) + 1
        return {
            "completed": len(lat), "failed": sum(1 for r in self.done if r.status != 0),
            "failed_by_status": fails,
            "bead_steps": self.bead_steps, "span_s": span,
            "bead_solves_per_s": self.bead_steps / span if span > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat else None,
            "ticks": self.ticks,
        }


def poisson_arrivals(rng, n: int, rate: float) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (per second)."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
