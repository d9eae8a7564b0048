"""Continuous-batching simulation server.

Requests (a mixture, a lattice and grid, an initial field) arrive over time.
A request is admitted as soon as its device memory fits the HBM budget and
a slot is free; from then on it shares the GPU with every other admitted
request: each tick advances all active simulations with batched launches
(``fuglbm_step_many``): one per step per (component count, precision) for
D2Q9, four per step (the multi-pass kernels) per precision for D3Q19.
These units of work go longest-first onto
the least-loaded of a few HIP streams (default priority), so launches of
different groups run side by side on the CUs; then every simulation's residual is read
(``fuglbm_diagnostics``, on the stream that stepped it).  A simulation
retires when its residual R_K <= tol (K = steps per tick) or at its step
cap; its fields are read back and its memory returned, and waiting
requests are admitted.

Latency = finish - arrival, service = finish - admit, both wall clock.
"""
import heapq
import time
from dataclasses import dataclass, field

import numpy as np

from . import capi


@dataclass
class Request:
    rid: int
    comps: list
    T: float
    lattice: int
    shape: tuple
    rho: np.ndarray
    arrival: float = 0.0            # seconds after the server starts
    kij: object = None
    precision: int = capi.FP32_STORAGE
    tol: float = 1e-8
    max_steps: int = 200000
    # filled by the server
    admit_t: float = None
    finish_t: float = None
    steps: int = 0
    residual: float = None
    converged: bool = False
    status: int = 0
    result: dict = field(default=None, repr=False)

    @property
    def N(self):
        return len(self.comps)

    def nbytes(self):
        nx, ny, nz = (tuple(self.shape) + (1, 1))[:3]
        return capi.fields_bytes(self.N, self.lattice, self.precision, nx, ny, nz)

    def csu(self):
        return int(np.prod(self.shape)) * self.N * self.steps


class Server:
    def __init__(self, hbm_budget_bytes, chunk=200, max_active=64, kappa_ref=0.02,
                 keep_fields=False, stream=None, streams=6):
        import torch
        self.budget = int(hbm_budget_bytes)
        self.chunk = int(chunk)
        self.max_active = int(max_active)
        self.kappa_ref = kappa_ref
        self.keep_fields = keep_fields
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.streams = [self.stream] + [torch.cuda.Stream() for _ in range(max(0, streams - 1))]
        self.used = 0
        self.done = []

    # -- lifecycle of one request --------------------------------------
    def _admit(self, req, now):
        mix = capi.Mixture.from_components(req.comps, req.T, req.kij, kappa_ref=self.kappa_ref)
        sim = capi.Simulation(mix, req.lattice, req.precision, req.shape, req.rho,
                              stream=self.stream)
        sim.diagnostics()                  # snapshot for the first residual
        req.admit_t = now
        self.used += req.nbytes()
        return dict(req=req, mix=mix, sim=sim)

    def _retire(self, slot, now, status=0):
        req, sim = slot["req"], slot["sim"]
        if self.keep_fields and status == 0:
            req.result = dict(populations=sim.read_populations(),
                              rho=sim.read_moments(velocity=False)["rho"])
        req.finish_t = now
        req.status = status
        sim.close()
        slot["mix"].close()
        self.used -= req.nbytes()
        self.done.append(req)

    def run(self, requests, clock=time.perf_counter, progress=None):
        """Serve `requests` (their `arrival` offsets are honoured in wall
        clock) until all are finished.  Returns the finished requests.
        `progress(t, active, waiting, done)` is called after every tick."""
        pending = [(r.arrival, r.rid, r) for r in requests]
        heapq.heapify(pending)
        waiting = []          # arrived, not admitted (FIFO)
        active = []
        t0 = clock()
        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0][0] <= now:
                waiting.append(heapq.heappop(pending)[2])
            # admission: FIFO, by HBM budget and slots
            while waiting and len(active) < self.max_active:
                req = waiting[0]
                if req.nbytes() > self.budget:
                    waiting.pop(0)
                    req.status = -1               # can never fit
                    req.finish_t = now
                    self.done.append(req)
                    continue
                if self.used + req.nbytes() > self.budget:
                    break
                waiting.pop(0)
                try:
                    active.append(self._admit(req, clock() - t0))
                except capi.FuglbmError as e:      # rejected input: fails alone
                    req.status = e.status
                    req.finish_t = clock() - t0
                    self.done.append(req)
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.05, pending[0][0] - (clock() - t0))))
                continue
            # one tick: every active simulation advances `chunk` steps; units
            # of work (a batched D2Q9 group of one component count and
            # precision, a batched D3Q19 group of one precision) go onto the
            # streams
            groups = {}
            for s in active:
                r = s["req"]
                key = (r.lattice, r.N if r.lattice == capi.D2Q9 else 0, r.precision)
                groups.setdefault(key, []).append(s)
            units = list(groups.values())
            # longest-first onto the least-loaded stream (work ~ CSU per step)
            cost = lambda u: sum(int(np.prod(s["req"].shape)) * s["req"].N *
                                 (19 if s["req"].lattice != capi.D2Q9 else 9) for s in u)
            load = [0] * len(self.streams)
            for unit in sorted(units, key=cost, reverse=True):
                k = min(range(len(load)), key=load.__getitem__)
                load[k] += cost(unit)
                st = self.streams[k]
                # ENONFINITE: a member with a sticky error was skipped; the
                # residual read below retires it alone
                rc = capi.fuglbm_step_many([s["sim"] for s in unit], self.chunk, st)
                if rc not in (0, 5):
                    capi.check(rc)
            still = []
            for s in active:
                req = s["req"]
                d = s["sim"].diagnostics()
                req.steps = d["step"]
                req.residual = d["residual"]
                if d["rc"] != 0:
                    self._retire(s, clock() - t0, status=d["rc"])
                elif req.residual <= req.tol:
                    req.converged = True
                    self._retire(s, clock() - t0)
                elif req.steps >= req.max_steps:
                    self._retire(s, clock() - t0)
                else:
                    still.append(s)
            active = still
            if progress is not None:
                progress(clock() - t0, len(active), len(waiting), len(self.done))
        return self.done


def latency_stats(done):
    """Time-to-equilibrium statistics over the requests that converged
    (R_K <= tol); a request retired at its step cap is counted as capped,
    not converged, and enters no percentile; failed requests (non-zero
    status) are counted apart."""
    conv = [r for r in done if r.status == 0 and r.converged]
    capped = [r for r in done if r.status == 0 and not r.converged]
    failed = [r for r in done if r.status != 0]
    out = dict(requests=len(done), converged=len(conv), capped=len(capped), failed=len(failed))
    if conv:
        lat = np.array([r.finish_t - r.arrival for r in conv])
        svc = np.array([r.finish_t - r.admit_t for r in conv])
        steps = np.array([r.steps for r in conv])
        out.update(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                   service_p50_s=float(np.percentile(svc, 50)),
                   service_p99_s=float(np.percentile(svc, 99)),
                   steps_p50=int(np.percentile(steps, 50)), steps_max=int(steps.max()))
    if capped:
        out["capped_residual_max"] = float(max(r.residual for r in capped))
    return out


def pool_requests(states, count, rate_hz, seed=5, precision=capi.FP32_STORAGE, tol=1e-8,
                  max_steps=200000, max_n2d=None, max_n3d=None, indices=None):
    """Requests from the stored serving pool (the first `count`, or the pool
    entries `indices` in that order), Poisson arrivals at `rate_hz`."""
    from inputs import fields as Fi
    from .batch import _Comp
    comps_all = [_Comp(**c) for c in states["components"]]
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    pool = states["requests"]
    picked = [(k, pool[k]) for k in indices] if indices is not None else list(enumerate(pool[:count]))
    for k, q in picked:
        t += rng.exponential(1.0 / rate_hz)
        N = q["N"]
        n = q["n"]
        if q["lattice"] == "D2Q9":
            if max_n2d:
                n = min(n, max_n2d)
            rho = Fi.slab(n, n, q["rho_V"], q["rho_L"], q["S_V"])
            lat, shape = capi.D2Q9, (n, n)
        else:
            if max_n3d:
                n = min(n, max_n3d)
            rho = Fi.slab(n, n, q["rho_V"], q["rho_L"], q["S_V"], nz=n)
            lat, shape = capi.D3Q19, (n, n, n)
        out.append(Request(k, comps_all[:N], q["T"], lat, shape, rho, arrival=t,
                           precision=precision, tol=tol, max_steps=max_steps))
    return out
