"""Continuous-batching request loop for spin-glass simulation jobs.

Requests (model, L, temperature, sweeps, seed) arrive over time.  A request
is admitted when a slot is free and its device arena fits in the remaining
HBM budget; admitted jobs join the running batch at the next period boundary
and share one fused sweep launch per period with every other resident job
(their lattices and wheel states stay on the device between periods).  Each
job carries its own sweep budget, so it stops exactly after its requested
number of sweeps; it is then measured, exported and released, and its memory
and slot go to the next waiting request.  A job's result does not depend on
which other jobs shared its launches (the random numbers of every site are
fixed by the job's own seed, copy, site and sweep).

The loop runs in wall-clock time and records, per request, the arrival,
admission and completion times; latency = completion - arrival.
"""
from __future__ import annotations

import dataclasses
import hashlib
import time
from collections import deque
from typing import Optional

import numpy as np

from . import binding as B
from . import inputs

def spins_fingerprint(spins: np.ndarray) -> int:
    """64-bit BLAKE2b fingerprint of the canonical spin bytes of a job."""
    return int.from_bytes(hashlib.blake2b(np.ascontiguousarray(spins).tobytes(),
                                          digest_size=8).digest(), "little")


@dataclasses.dataclass
class Request:
    rid: int
    model: str          # "ising" (Metropolis) or "potts" (heat bath)
    L: int
    T: float
    sweeps: int
    seed: int
    arrival: float = 0.0           # seconds after the start of the stream
    # filled in by the server
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    E: Optional[np.ndarray] = None  # energy of replica 0 and 1
    Q: Optional[int] = None         # overlap of the two replicas
    spins_hash: Optional[int] = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival

    def updates(self) -> int:
        return 2 * self.L ** 3 * self.sweeps


def make_job(ctx, req: Request, arena=None) -> B.Job:
    model = B.ISING if req.model == "ising" else B.POTTS
    algo = B.METROPOLIS if req.model == "ising" else B.HEATBATH
    inst = inputs.make_instance(req.model, req.L, 1, 2, 1, req.seed)
    return B.Job(ctx, model, algo, req.L, [1.0 / req.T], inst["J"], inst["spins"],
                 inst["wheels"], n_samples=1, n_replicas=2, arena=arena)


def job_bytes(req: Request) -> int:
    model = B.ISING if req.model == "ising" else B.POTTS
    algo = B.METROPOLIS if req.model == "ising" else B.HEATBATH
    return B.job_bytes(B.Spec(model, algo, 4, req.L, 1, 2, 1, 0))


def finish(job: B.Job, req: Request):
    E, Q = job.measure()
    req.E = E
    req.Q = int(Q[0])
    req.spins_hash = spins_fingerprint(job.spins())


class DeviceBackend:
    """Jobs and batches of libsg on one GPU (arenas are torch tensors)."""

    def __init__(self, ctx, stream=None):
        self.ctx = ctx
        self.stream = stream

    def new_batch(self):
        return B.Batch(self.ctx)

    def job_bytes(self, req):
        return job_bytes(req)

    def create(self, req):
        import torch
        arena = torch.empty(job_bytes(req), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        return make_job(self.ctx, req, arena)

    def run(self, batch, n):
        import torch
        batch.run(n, self.stream)
        torch.cuda.synchronize()

    def finish(self, job, req):
        finish(job, req)


class Server:
    """Admission by slots and HBM budget + continuous batching."""

    def __init__(self, backend, hbm_budget: int, max_slots: int = 512, period: int = 500):
        self.be = backend
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.period = period
        self.batch = backend.new_batch()
        self.used = 0
        self.peak_used = 0
        self.peak_slots = 0
        self.active = {}   # rid -> (job, req, bytes)
        self.pending = deque()
        self.done = []
        self.periods = 0

    def _admit(self, now: float):
        while self.pending and len(self.active) < self.max_slots:
            req = self.pending[0]
            nb = self.be.job_bytes(req)
            if nb > self.budget:
                raise RuntimeError(f"request {req.rid} needs {nb} bytes, budget {self.budget}")
            if self.used + nb > self.budget:
                break
            self.pending.popleft()
            job = self.be.create(req)
            self.batch.add(job)
            self.batch.set_budget(job, req.sweeps)
            self.used += nb
            self.peak_used = max(self.peak_used, self.used)
            req.t_admit = now
            self.active[req.rid] = (job, req, nb)
            self.peak_slots = max(self.peak_slots, len(self.active))

    def _harvest(self, now: float):
        for rid in [r for r, (job, req, nb) in self.active.items()
                    if job.sweeps_done() >= req.sweeps]:
            job, req, nb = self.active.pop(rid)
            self.be.finish(job, req)
            req.t_done = now
            self.batch.remove(job)
            job.close()
            self.used -= nb
            self.done.append(req)

    def serve(self, requests, clock=time.perf_counter, sleep=time.sleep):
        """Run a stream of requests (any order; served by arrival) to completion."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = clock()
        i = 0
        while i < len(reqs) or self.pending or self.active:
            now = clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                self.pending.append(reqs[i])
                i += 1
            self._admit(now)
            if self.active:
                # one period: every resident job advances min(period, its budget)
                n = min(self.period, max(req.sweeps - job.sweeps_done()
                                         for job, req, _ in self.active.values()))
                self.be.run(self.batch, n)
                self.periods += 1
                self._harvest(clock() - t0)
            elif i < len(reqs):
                sleep(max(0.0, min(0.01, reqs[i].arrival - (clock() - t0))))
        return self.done


def poisson_stream(n_jobs: int, rate: float, seed: int = 5, sweeps_lo: float = 3.0,
                   sweeps_hi: float = 5.0, sizes=(8, 16, 24, 32, 48), t_range=(0.7, 1.6),
                   seed0: int = 5000):
    """Requests with exponential inter-arrival times (rate per second); model
    Ising or Potts with probability 1/2, L uniform in `sizes`, T uniform in
    t_range, sweeps = floor(10^U[sweeps_lo, sweeps_hi]), job seed seed0 + j
    (parameters from inputs.job_stream)."""
    return [Request(**p) for p in inputs.job_stream(n_jobs, rate, seed, sweeps_lo, sweeps_hi,
                                                      sizes, t_range, seed0)]


def summary(done, wall: float):
    lat = np.array([r.latency for r in done])
    upd = sum(r.updates() for r in done)
    return {"jobs": len(done), "wall_s": round(wall, 3),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "jobs_per_s": round(len(done) / wall, 3),
            "updates_per_ns": round(upd / (wall * 1e9), 3)}
