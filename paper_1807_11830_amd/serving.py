"""Continuous-batching reconstruction server for CG-SENSE requests.

Requests (one 2D slice each: size, coil count, acceleration, iteration
count) arrive over time.  The scheduler admits them first-in first-out into
an executor's slots as slots and device memory free up, advances every
admitted solve by one CG iteration per step, and retires finished ones:
requests that arrive while others run join the next step, so their work
overlaps on the device (continuous batching, not a queue in front of a
single solver).  Latency is arrival -> result ready.

Executors:
* :class:`EngineExecutor` - the library's slot-table engine (batched fused
  E^H E and CG-update launches per size group), with plans pooled per
  (size, coils, mask) and rebound to each request's maps;
* :class:`SerialExecutor` - one solve at a time with the plain
  ``Plan.cg`` path (whole-solve graph), the baseline;
* any object with ``admit(req) -> bool``, ``step()``, ``poll() -> ids``
  and ``release(req)`` (the CPU tests drive the scheduler with a fake one
  on a virtual clock).
"""
from __future__ import annotations

import math
import time
from collections import defaultdict, deque
from dataclasses import dataclass, field
from typing import Any, Callable

import numpy as np


@dataclass
class Request:
    id: int
    arrival: float
    n: int
    ncoils: int
    accel: int
    iters: int
    seed: int | None = None  # inputs drawn from this seed (None: per-class inputs)
    payload: Any = None
    admitted: float = math.nan
    finished: float = math.nan
    result: Any = None


@dataclass
class RunStats:
    n: int
    makespan: float
    throughput: float
    p50: float
    p99: float
    mean: float
    max_inflight: int
    steps: int = 0
    extra: dict = field(default_factory=dict)


class Scheduler:
    """FIFO admission, one executor step per turn, retirement by poll."""

    def __init__(self, executor, clock: Callable[[], float] = None, sleep: Callable[[float], None] = None):
        self.ex = executor
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep

    def run(self, requests):
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.id)))
        queue = deque()
        inflight = {}
        max_inflight = 0
        steps = 0
        while pending or queue or inflight:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            while queue:
                r = queue[0]
                if not self.ex.admit(r):
                    if not inflight:
                        raise RuntimeError(f"request {r.id} can never be admitted (too large for the budget)")
                    break
                r.admitted = now()
                inflight[r.id] = r
                queue.popleft()
            max_inflight = max(max_inflight, len(inflight))
            if inflight:
                self.ex.step()
                steps += 1
                for rid in self.ex.poll():
                    r = inflight.pop(rid)
                    r.finished = now()
                    self.ex.release(r)
            elif pending:
                self.sleep(max(0.0, pending[0].arrival - now()))
        return stats(requests, max_inflight, steps)


def stats(requests, max_inflight=0, steps=0) -> RunStats:
    lat = np.array([r.finished - r.arrival for r in requests])
    span = max(r.finished for r in requests) - min(r.arrival for r in requests)
    return RunStats(n=len(requests), makespan=float(span), throughput=len(requests) / span,
                    p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                    mean=float(lat.mean()), max_inflight=max_inflight, steps=steps)


# ---------------------------------------------------------------------------
# GPU executors
# ---------------------------------------------------------------------------

class InputBank:
    """Seeded synthetic inputs, resident on the GPU.

    Every request of a stream carries its own sub-seed (SeedSequence
    children of the stream seed): its coil maps are the Gaussian-bump set
    rotated by an angle drawn from that seed, its image is a phantom drawn
    from it and its noise is drawn from it, so every request in flight reads
    its own maps and k-space buffers (no request shares an input buffer with
    another).  The mask is the variable-density mask of the request's
    (size, acceleration) class.  Requests without a seed (hand-made test
    requests) use per-class inputs: maps per (n, coils), k-space per
    (n, coils, accel)."""

    def __init__(self, device="cuda:0", n_centre=24):
        import torch

        from . import synth

        self.torch = torch
        self.synth = synth
        self.device = torch.device(device)
        self.n_centre = n_centre
        self.maps, self.masks, self.y = {}, {}, {}
        self.req = {}  # (seed, n, coils, accel) -> (maps, y) of one seeded request
        self.eplans = {}  # (n, coils, accel) -> plan that forms y = E x

    @staticmethod
    def _key(r):
        return (r.seed, r.n, r.ncoils, r.accel)

    def mask(self, n, accel):
        k = (n, accel)
        if k not in self.masks:
            self.masks[k] = self.synth.mask_variable_density(n, float(accel), self.n_centre)
        return self.masks[k]

    def coil_maps(self, n, c):
        k = (n, c)
        if k not in self.maps:
            m = self.synth.coil_maps2d(n, c).astype(np.complex64)
            self.maps[k] = self.torch.from_numpy(m).to(self.device)
        return self.maps[k]

    def _kspace_of(self, maps, img, noise, n, accel):
        from .sense import Plan

        torch = self.torch
        mask = self.mask(n, accel)
        k = (n, maps.shape[0], accel)
        if k not in self.eplans:
            self.eplans[k] = Plan(maps, mask)
        plan = self.eplans[k]
        plan.set_maps(maps)
        y = plan.E(img)
        y += torch.from_numpy(noise * mask[None, None, :, None]).to(self.device)
        return y

    def kspace(self, n, c, accel):
        k = (n, c, accel)
        if k not in self.y:
            img = self.torch.from_numpy(self.synth.phantom2d(n).astype(np.complex64)[None]).to(self.device)
            noise = self.synth.complex_noise((1, c, n, n)).astype(np.complex64)
            self.y[k] = self._kspace_of(self.coil_maps(n, c), img, noise, n, accel)
        return self.y[k]

    def _draw(self, r):
        """Host arrays of request r from its own seed (maps, image, noise)."""
        rng = np.random.default_rng(r.seed)
        rot = float(rng.uniform(0.0, 2.0 * np.pi))
        maps = self.synth.coil_maps2d(r.n, r.ncoils, rotation=rot).astype(np.complex64)
        img = self.synth.phantom2d(r.n, seed=int(rng.integers(0, 2**31))).astype(np.complex64)[None]
        noise = self.synth.complex_noise((1, r.ncoils, r.n, r.n), seed=int(rng.integers(0, 2**31)))
        return maps, img, noise.astype(np.complex64)

    def inputs(self, r):
        """(maps, y) of request r on the GPU."""
        if r.seed is None:
            return self.coil_maps(r.n, r.ncoils), self.kspace(r.n, r.ncoils, r.accel)
        if self._key(r) not in self.req:
            self._make([r])
        return self.req[self._key(r)]

    def _make(self, reqs):
        import concurrent.futures as cf

        torch = self.torch
        todo, seen = [], set()
        for r in reqs:
            if r.seed is not None and self._key(r) not in self.req and self._key(r) not in seen:
                seen.add(self._key(r))
                todo.append(r)
        # numpy draws run in a thread pool (they release the GIL); uploads
        # and the forward model run here, in request order
        with cf.ThreadPoolExecutor(max_workers=8) as ex:
            for r, (m, img, noise) in zip(todo, ex.map(self._draw, todo)):
                maps = torch.from_numpy(m).to(self.device)
                y = self._kspace_of(maps, torch.from_numpy(img).to(self.device), noise, r.n, r.accel)
                self.req[self._key(r)] = (maps, y)

    def prepare(self, requests):
        self._make(list(requests))
        for r in requests:
            if r.seed is None:
                self.kspace(r.n, r.ncoils, r.accel)
        self.torch.cuda.synchronize()

    def drop(self, requests):
        """Free the per-request inputs of these requests."""
        for r in requests:
            self.req.pop(self._key(r), None)

    def close(self):
        for p in self.eplans.values():
            p.close()
        self.eplans.clear()

    def nbytes(self):
        """Device bytes of all resident inputs."""
        tot = 0
        for m, y in self.req.values():
            tot += m.numel() * m.element_size() + y.numel() * y.element_size()
        return tot


class PlanPool:
    """Idle plans per (n, coils, accel): creating a plan allocates device
    memory, so finished requests hand theirs back for the next request of
    the same class (rebound to that request's maps)."""

    def __init__(self, bank: InputBank):
        self.bank = bank
        self.idle = defaultdict(list)
        self.created = 0

    def get(self, r, maps):
        from .sense import Plan

        key = (r.n, r.ncoils, r.accel)
        if self.idle[key]:
            plan = self.idle[key].pop()
            plan.set_maps(maps)
            return plan
        self.created += 1
        return Plan(maps, self.bank.mask(r.n, r.accel))

    def put(self, r, plan):
        self.idle[(r.n, r.ncoils, r.accel)].append(plan)

    def close(self):
        for lst in self.idle.values():
            for p in lst:
                p.close()
        self.idle.clear()


def footprint(r, plan_bytes: int) -> int:
    """Device bytes a request holds while admitted: its plan, its own
    k-space and maps (C images each) and its output image."""
    return plan_bytes + 8 * r.n * r.n * (2 * r.ncoils + 1)


class EngineExecutor:
    def __init__(self, bank: InputBank, budget_bytes: int, max_slots: int):
        from .sense import Engine, device_bytes

        self.bank = bank
        self.pool = PlanPool(bank)
        self.engine = Engine(budget_bytes, max_slots, device=bank.device)
        self.device_bytes = device_bytes
        self.slot_req = {}

    def admit(self, r) -> bool:
        torch = self.bank.torch
        fp = footprint(r, self.device_bytes(r.n, r.n, r.ncoils, 1))
        st = self.engine.stats()
        if len(self.slot_req) >= self.engine.max_slots or st["used"] + fp > st["budget"]:
            return False
        maps, y = self.bank.inputs(r)
        plan = self.pool.get(r, maps)
        x = torch.empty((1, r.n, r.n), dtype=torch.complex64, device=self.bank.device)
        slot = self.engine.admit(plan, y, x, r.iters, footprint=fp)
        if slot is None:
            self.pool.put(r, plan)
            return False
        r.payload = (plan, x, slot)
        self.slot_req[slot] = r.id
        return True

    def step(self):
        self.engine.step()

    def poll(self):
        return [self.slot_req.pop(s) for s in self.engine.poll()]

    def release(self, r):
        plan, x, slot = r.payload
        r.result = x
        self.pool.put(r, plan)
        r.payload = None

    def close(self):
        self.engine.sync()
        self.engine.close()
        self.pool.close()


class SerialExecutor:
    """One solve at a time through Plan.cg (the plain path).  Every request
    brings new buffers, so a captured whole-solve graph would be captured
    again for each one; the solves are launched eagerly instead."""

    def __init__(self, bank: InputBank, graphs: bool = False):
        self.bank = bank
        self.pool = PlanPool(bank)
        self.graphs = graphs
        self.cur = None
        self.event = None

    def admit(self, r) -> bool:
        torch = self.bank.torch
        if self.cur is not None:
            return False
        maps, y = self.bank.inputs(r)
        plan = self.pool.get(r, maps)
        plan.set_graphs(self.graphs)
        x = torch.empty((1, r.n, r.n), dtype=torch.complex64, device=self.bank.device)
        plan.cg(y, r.iters, out=x, sync=False)
        self.event = torch.cuda.Event()
        self.event.record()
        r.payload = (plan, x)
        self.cur = r
        return True

    def step(self):
        pass

    def poll(self):
        if self.cur is not None and self.event.query():
            r, self.cur = self.cur, None
            return [r.id]
        return []

    def release(self, r):
        plan, x = r.payload
        r.result = x
        self.pool.put(r, plan)
        r.payload = None

    def close(self):
        self.pool.close()


def make_requests(n_requests, rate, iters=25, seed=None, **kw):
    """Poisson request stream (synth.request_stream) as Request objects."""
    from . import synth

    kw = dict(kw)
    if seed is not None:
        kw["seed"] = seed
    return [Request(d["id"], d["arrival"], d["n"], d["ncoils"], d["accel"], iters, seed=d["seed"])
            for d in synth.request_stream(n_requests, rate, **kw)]
