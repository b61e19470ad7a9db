"""Serving form: Newton-step solve requests from many concurrent simulations.

A request names a simulation and a right-hand side (a new seeded F, G for
that simulation's element matrices).  Simulations are admitted to the
device under a byte budget; an admitted simulation keeps its FP64 element
matrices, its low-precision element factors and its BILU(0) factors
resident, so a later request for it needs only the right-hand-side path
(condensation of F, assembly of R, GMRES, back-substitution, FP64
refinement).  A request for a simulation that is not resident first
condenses and factors it.

Continuous batching: every request runs on one of several HIP streams
("slots"); a request that arrives while others are on the device starts as
soon as a slot is free and its memory can be admitted, so requests overlap
on the GPU.  Idle resident simulations are evicted least-recently-used when
the budget is needed.  Requests of one simulation run one at a time.
"""
import math
import time
from collections import OrderedDict, deque
from dataclasses import dataclass

import numpy as np
import torch

from . import api
from ._lib import F32
from .batch import Simulation


@dataclass
class Request:
    rid: int
    sim: int
    rhs: int
    arrival: float           # seconds after the start of the run
    start: float = None
    done: float = None
    hit: bool = None
    rho: float = None
    iters: int = None
    eager_steps: int = 0
    error: str = None
    uhat: torch.Tensor = None
    z: torch.Tensor = None

    @property
    def latency(self):
        return self.done - self.arrival


def poisson_requests(seed, n_requests, rate, n_sims):
    """Seeded request stream: exponential gaps at `rate` per second, the
    simulation drawn uniformly, right-hand side ids counting per simulation
    from 1 (id 0 is the simulation's initial right-hand side)."""
    from synth.philox import philox4x32_10
    idx = np.arange(n_requests, dtype=np.uint64)
    x0, x1, _, _ = philox4x32_10(idx, 0, 0xFFFFFFFD, 0, seed & 0xFFFFFFFF, seed >> 32)
    u = (x0.astype(np.float64) + 1.0) / 4294967296.0          # (0, 1]
    gaps = -np.log(u) / rate
    arrivals = np.cumsum(gaps) - gaps[0]
    sims = (x1 % np.uint32(n_sims)).astype(int)
    count = [0] * n_sims
    out = []
    for i in range(n_requests):
        s = int(sims[i])
        count[s] += 1
        out.append(Request(i, s, count[s], float(arrivals[i])))
    return out


class _Slot:
    def __init__(self, device):
        self.stream = torch.cuda.Stream()
        # a context per slot: a device error latched by a request fails that
        # request alone
        self.ctx = api.Context(device)
        self.event = None
        self.req = None
        self.sums_host = None


class Server:
    """Request loop over `cases` (one simulation per case).

    Every simulation's mesh and GMRES workspaces are created up front (small
    and fixed); its per-solve arrays (FP64 element matrices, factors, trace
    system, vectors) live in a byte arena while it is resident.  Admission
    takes the smallest free arena that fits, else a new one within the
    budget, else evicts idle residents (least recently used first), whose
    arenas go to the free list rather than back to the allocator, so the
    request loop itself allocates and frees no device memory once the pool
    has formed."""

    def __init__(self, ctx, cases, seed, budget_bytes=200e9, n_slots=4, prec=F32, restart=100, tol=1e-8,
                 n_refine=1, keep_results=False):
        self.ctx, self.cases, self.seed = ctx, list(cases), seed
        self.budget = float(budget_bytes)
        self.prec, self.restart, self.tol, self.n_refine = prec, restart, tol, n_refine
        self.keep = keep_results
        dev = torch.cuda.current_device()
        self.slots = [_Slot(dev) for _ in range(n_slots)]
        self.sims = [Simulation(ctx, c, seed, prec=prec, restart=restart, n_refine=n_refine, tol=tol,
                                allocate=False) for c in self.cases]
        self.static_bytes = sum(s.static_bytes() for s in self.sims)
        self.need = [s.arena_bytes() for s in self.sims]
        self.arena_budget = self.budget - self.static_bytes
        for sid, nb in enumerate(self.need):
            if nb > self.arena_budget:
                raise ValueError(f"simulation {sid} needs {nb / 1e9:.1f} GB > budget")
        self.resident = OrderedDict()      # sim id -> None, least recently used first
        self.free = []                     # idle arenas
        self.allocated = 0                 # bytes of all arenas (resident and idle)
        self.busy = set()
        self.stats = {"hits": 0, "misses": 0, "evictions": 0, "arenas_allocated": 0, "arenas_reused": 0,
                      "arenas_dropped": 0, "failed": 0}

    # -- residency ------------------------------------------------------------
    def _best_free(self, need):
        fits = [i for i, a in enumerate(self.free) if a.numel() >= need]
        return min(fits, key=lambda i: self.free[i].numel()) if fits else None

    def _can_admit(self, sid):
        if sid in self.resident:
            return True
        need = self.need[sid]
        if self._best_free(need) is not None or self.allocated + need <= self.arena_budget:
            return True
        idle = sum(self.sims[s].arena.numel() for s in self.resident if s not in self.busy)
        free = sum(a.numel() for a in self.free)
        return self.allocated - idle - free + need <= self.arena_budget

    def _evict(self, s):
        del self.resident[s]
        self.free.append(self.sims[s].detach())
        self.stats["evictions"] += 1

    def _admit(self, sid):
        need = self.need[sid]
        pick = self._best_free(need)
        if pick is None and self.allocated + need > self.arena_budget:
            for s in [s for s in self.resident if s not in self.busy]:
                self._evict(s)
                pick = self._best_free(need)
                if pick is not None or self.allocated + need <= self.arena_budget:
                    break
        if pick is not None:
            arena = self.free.pop(pick)
            self.stats["arenas_reused"] += 1
        else:
            # drop idle arenas (smallest first) until a new one fits
            self.free.sort(key=lambda a: a.numel())
            while self.free and self.allocated + need > self.arena_budget:
                self.allocated -= self.free.pop(0).numel()
                self.stats["arenas_dropped"] += 1
            assert self.allocated + need <= self.arena_budget
            arena = torch.empty(need, dtype=torch.uint8, device="cuda")
            self.allocated += need
            self.stats["arenas_allocated"] += 1
        self.sims[sid].attach(arena)
        self.resident[sid] = None
        return self.sims[sid]

    def _bind(self, sim, ctx):
        sim.ctx = ctx
        for g in sim.gm:
            g.ctx = ctx

    # -- one request on one slot ----------------------------------------------
    def _launch(self, slot, req, now):
        sid = req.sim
        req.start = now
        with torch.cuda.stream(slot.stream):
            if sid in self.resident:
                sim = self.sims[sid]
                self.resident.move_to_end(sid)
                req.hit = True
                self.stats["hits"] += 1
                self._bind(sim, slot.ctx)
                sim.set_rhs(req.rhs)
                sim.enqueue_rhs()
            else:
                sim = self._admit(sid)
                req.hit = False
                self.stats["misses"] += 1
                self._bind(sim, slot.ctx)
                sim.generate(req.rhs)
                # factor, then the same right-hand-side path as a hit: a
                # request's result does not depend on whether it hit
                sim.enqueue_factor()
                sim.enqueue_rhs()
            if slot.sums_host is None or slot.sums_host.shape != sim.sums.shape:
                slot.sums_host = torch.empty(sim.sums.shape, dtype=torch.float64, pin_memory=True)
            slot.sums_host.copy_(sim.sums, non_blocking=True)
            if self.keep:
                req.uhat = sim.uhat.clone()
                req.z = sim.z.clone()
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        self.busy.add(sid)
        slot.event, slot.req = ev, req

    def _complete(self, slot, now):
        req = slot.req
        req.done = now
        sim = self.sims[req.sim]
        try:
            with torch.cuda.stream(slot.stream):
                slot.ctx.sync_status()
        except api.IedgError as err:
            # this request fails alone; its simulation's state is suspect
            req.error = str(err)
            req.rho = float("nan")
            self.stats["failed"] += 1
            self.busy.discard(req.sim)
            if req.sim in self.resident:
                self._evict(req.sim)
            slot.event = slot.req = None
            return
        sums = slot.sums_host.tolist()
        rho = Simulation._rho(sums[-1])
        if not rho <= self.tol:
            # rare: the captured refinement was not enough; continue eagerly
            with torch.cuda.stream(slot.stream):
                res = sim.finish(sums=sums)
                if self.keep:
                    req.uhat = sim.uhat.clone()
                    req.z = sim.z.clone()
                torch.cuda.current_stream().synchronize()
            rho = res.rho_hist[-1]
            req.eager_steps = res.eager_steps
            req.iters = sum(res.iters)
            req.done = time.perf_counter() - self._t0
        req.rho = rho
        req.iters = sum(g.read()["iters"] for g in sim.gm) if req.iters is None else req.iters
        self.busy.discard(req.sim)
        slot.event = slot.req = None

    # -- the loop ---------------------------------------------------------------
    def run(self, requests, real_time=True, progress=None, every=250):
        """Serve `requests` (sorted by arrival).  real_time: arrivals follow
        the wall clock; otherwise every request is available at once.
        progress(done, total) is called after every `every` completions."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = []
        done = []
        self._t0 = time.perf_counter()
        while pending or queue or any(s.req for s in self.slots):
            now = time.perf_counter() - self._t0
            while pending and (not real_time or pending[0].arrival <= now):
                queue.append(pending.popleft())
            progressed = False
            for slot in self.slots:
                if slot.req is not None and slot.event.query():
                    r = slot.req
                    self._complete(slot, time.perf_counter() - self._t0)
                    done.append(r)
                    progressed = True
                    if progress is not None and len(done) % every == 0:
                        progress(len(done), len(requests))
            for slot in self.slots:
                if slot.req is not None:
                    continue
                pick = None
                for i, r in enumerate(queue):
                    if r.sim not in self.busy and self._can_admit(r.sim):
                        pick = i
                        break
                if pick is None:
                    break
                r = queue.pop(pick)
                self._launch(slot, r, time.perf_counter() - self._t0)
                progressed = True
            if not progressed:
                time.sleep(20e-6)
        return done

    def close(self):
        torch.cuda.synchronize()
        for sim in self.sims:
            sim.close()
        self.sims = []
        self.resident.clear()
        self.free.clear()
        self.allocated = 0


def summarize(done, elapsed=None):
    ok = [r for r in done if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    span = elapsed if elapsed is not None else max(r.done for r in done) - min(r.arrival for r in done)
    return {"requests": len(done), "solves_per_s": len(done) / span if span > 0 else float("nan"),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "hit_rate": sum(1 for r in done if r.hit) / len(done),
            "max_rho": max(r.rho for r in ok), "failed": len(done) - len(ok)}
