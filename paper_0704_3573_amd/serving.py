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

The loop never synchronises the whole device.  Jobs are created from their
seed alone (the library generates the instance) by a worker thread on a
stream of its own, while periods run; a period's end is a HIP event the loop
polls; while the membership stays the same, a second period is enqueued
behind the running one, so the device does not wait for the host.  Jobs of
one period differ widely in the device time of a sweep (an L = 48 Potts copy
against an L = 8 Ising one), so in each period every job runs about the same
device time rather than the same number of sweeps: a period would otherwise
last as long as its slowest job while the others' compute units idle.

A request can be cancelled (Server.cancel) while it waits, while its job
is being created or while it is resident; a resident job leaves the batch at
the next period boundary, and the others continue unchanged.

The loop runs in wall-clock time and records, per request, the arrival,
admission and completion times; latency = completion - arrival.  An optional
wall-clock cap stops it with work still in flight (for streams far longer
than a measurement); the sweeps performed by then are counted.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import hashlib
import threading
import time
import collections
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
    cancelled: bool = False

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival

    def updates(self) -> int:
        return 2 * self.L ** 3 * self.sweeps


def _model_algo(req: Request):
    return ((B.ISING, B.METROPOLIS) if req.model == "ising" else (B.POTTS, B.HEATBATH))


def make_job(ctx, req: Request, arena=None, stream=None) -> B.Job:
    """The job of a request, created from its seed alone (two replicas, one
    temperature); its inputs are those of inputs.make_instance."""
    model, algo = _model_algo(req)
    return B.Job(ctx, model, algo, req.L, [1.0 / req.T], n_samples=1, n_replicas=2,
                 arena=arena, stream=stream, seed=req.seed)


def sweep_cost(req: Request) -> float:
    """Relative device time of one sweep of a request's job: draws per lane
    per sweep (min(8, L) rows of L sites per wheel, shared by the lanes of
    the wheel: four for the Potts model at L = 8..32, two at L = 40, 48)
    times the cost of a draw per lane (a Potts heat-bath update about eight
    Ising Metropolis ones, from the measured per-lane rates of the two
    kernels).  Only a scheduling estimate: it sets how many sweeps each job
    runs in a period."""
    lanes = 1
    if req.model == "potts":
        lanes = 4 if req.L in (8, 16, 24, 32) else 2 if req.L in (40, 48) else 1
    return min(8, req.L) * req.L / lanes * (8.0 if req.model == "potts" else 1.0)


def job_bytes(req: Request) -> int:
    model, algo = _model_algo(req)
    return B.job_bytes(B.Spec(model, algo, 4, req.L, 1, 2, 1, 0))


def finish(job: B.Job, req: Request, stream=None):
    E, Q = job.measure(stream)
    req.E = E
    req.Q = int(Q[0])
    req.spins_hash = spins_fingerprint(job.spins(stream))


class DeviceBackend:
    """Jobs and batches of libsg on one GPU (arenas are torch tensors).

    Periods run on `stream` (a new non-blocking torch stream by default);
    jobs are created by `workers` threads, each on a creation stream of its
    own (a job's instance is generated on the host from its seed, then
    uploaded)."""

    def __init__(self, ctx, stream=None, workers=2):
        import torch
        self.ctx = ctx
        self.stream = stream if stream is not None else torch.cuda.Stream()
        # creation streams made here, on the caller's thread; each worker
        # thread takes one the first time it creates a job
        self._streams = [torch.cuda.Stream() for _ in range(workers)]
        self._local = threading.local()
        self._lock = threading.Lock()
        self.pool = cf.ThreadPoolExecutor(max_workers=workers)
        self.busy = []  # timing events around each period

    def new_batch(self):
        return B.Batch(self.ctx)

    def job_bytes(self, req):
        return job_bytes(req)

    def _create(self, req):
        import torch
        st = getattr(self._local, "stream", None)
        if st is None:
            with self._lock:
                st = self._local.stream = self._streams.pop()
        with torch.cuda.stream(st):
            arena = torch.empty(job_bytes(req), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
            return make_job(self.ctx, req, arena, st)

    def create_async(self, req):
        return self.pool.submit(self._create, req)

    @staticmethod
    def ready(handle) -> bool:
        return handle.done()

    @staticmethod
    def take(handle):
        return handle.result()

    def launch(self, batch, n):
        import torch
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(self.stream)
        batch.run(n, self.stream)
        t1.record(self.stream)
        self.busy.append((t0, t1))
        return t1

    def busy_seconds(self) -> float:
        """Device time of the periods launched so far (they run one after
        another on one stream), waiting for them."""
        total = 0.0
        for t0, t1 in self.busy:
            t1.synchronize()
            total += t0.elapsed_time(t1) * 1e-3
        return total

    @staticmethod
    def done(token) -> bool:
        return token.query()

    @staticmethod
    def wait(token):
        token.synchronize()

    def finish(self, job, req):
        finish(job, req, self.stream)

    def close(self):
        self.pool.shutdown(wait=True)


class Server:
    """Admission by slots and HBM budget + continuous batching."""

    def __init__(self, backend, hbm_budget: int, max_slots: int = 512, period: int = 64,
                 depth: int = 2):
        self.be = backend
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.period = period        # sweeps of the slowest resident job per period
        self.depth = depth          # periods in flight while the membership is unchanged
        self.batch = backend.new_batch()
        self.used = 0
        self.peak_used = 0
        self.peak_slots = 0
        self.active = {}            # rid -> (job, req, bytes)
        self.creating = deque()     # (req, handle, bytes), admission order
        self.pending = deque()
        self.inflight = deque()     # events of enqueued periods
        self.done = []
        self.periods = 0
        self.changes = 0            # membership changes (each re-plans the batch)
        self.cancelled = []         # requests cancelled before completion
        self._cancel = set()        # rids to cancel once arrived, created or resident
        self._cancelled_updates = 0
        self._caps = {}             # per-run cap last set, by rid
        self.host_s = collections.Counter()  # host seconds per loop step
        self.n = 1                  # sweeps per run (the largest per-run cap)

    def _admit(self):
        """Reserve memory and a slot for waiting requests (FIFO) and start
        creating their jobs."""
        while self.pending and len(self.active) + len(self.creating) < self.max_slots:
            req = self.pending[0]
            nb = self.be.job_bytes(req)
            if nb > self.budget:
                raise RuntimeError(f"request {req.rid} needs {nb} bytes, budget {self.budget}")
            if self.used + nb > self.budget:
                break
            self.pending.popleft()
            self.used += nb
            self.peak_used = max(self.peak_used, self.used)
            self.creating.append((req, self.be.create_async(req), nb))

    def _ready(self):
        return [c for c in self.creating if self.be.ready(c[1])]

    def cancel(self, rid) -> bool:
        """Cancel request rid: a waiting request is dropped, a job being
        created is released once created, a resident job leaves the batch at
        the next period boundary; none of them completes.  False if the
        request has already completed."""
        if any(r.rid == rid for r in self.done):
            return False
        for r in self.pending:
            if r.rid == rid:
                self.pending.remove(r)
                self._mark_cancelled(r)
                return True
        self._cancel.add(rid)
        return True

    def _mark_cancelled(self, req):
        req.cancelled = True
        self._cancel.discard(req.rid)
        self.cancelled.append(req)

    def _drop_cancelled(self):
        """Resident jobs cancelled since the last period boundary leave."""
        for rid in [r for r in self._cancel if r in self.active]:
            job, req, nb = self.active.pop(rid)
            self._caps.pop(rid, None)
            self._cancelled_updates += 2 * req.L ** 3 * job.sweeps_done()
            self.batch.remove(job)
            job.close()
            self.used -= nb
            self._mark_cancelled(req)

    def _join(self, ready, now):
        for c in ready:
            self.creating.remove(c)
            req, h, nb = c
            job = self.be.take(h)
            if req.rid in self._cancel:
                job.close()
                self.used -= nb
                self._mark_cancelled(req)
                continue
            self.batch.add(job)
            self.batch.set_budget(job, req.sweeps)
            req.t_admit = now
            self.active[req.rid] = (job, req, nb)
        self.peak_slots = max(self.peak_slots, len(self.active))

    def _finished(self):
        return [r for r, (job, req, nb) in self.active.items() if job.sweeps_done() >= req.sweeps]

    def _harvest(self, rids, now):
        for rid in rids:
            job, req, nb = self.active.pop(rid)
            self.be.finish(job, req)
            req.t_done = now
            self.batch.remove(job)
            job.close()
            self.used -= nb
            self.done.append(req)
            self._caps.pop(rid, None)
            self._cancel.discard(rid)  # completed before its cancellation took effect

    def _drain(self):
        if self.inflight:
            self.be.wait(self.inflight[-1])
            self.inflight.clear()

    def _set_caps(self):
        """Per-run caps after a membership change: the slowest resident job
        (by sweep_cost) runs `period` sweeps per period, every other job as
        many as take the same device time (its budget still stops it
        exactly).  The caps stay until the next change, so consecutive periods
        reuse the launch tables."""
        if not self.active:
            return
        slow = max(sweep_cost(req) for _, req, _ in self.active.values())
        self.n = 1
        for rid, (job, req, _) in self.active.items():
            cap = max(1, int(self.period * slow / sweep_cost(req)))
            if self._caps.get(rid) != cap:  # a library call only when it changes
                self.batch.set_period_cap(job, cap)
                self._caps[rid] = cap
            self.n = max(self.n, min(cap, req.sweeps))

    def _launch(self):
        self.inflight.append(self.be.launch(self.batch, self.n))
        self.periods += 1

    def release(self):
        """Release every job the server still holds (after serve() stopped at
        its wall-clock cap): the periods in flight are waited for and the
        jobs still being created are taken and closed."""
        self._drain()
        for req, h, nb in list(self.creating):
            self.be.take(h).close()
        self.creating.clear()
        for job, req, nb in list(self.active.values()):
            self.batch.remove(job)
            job.close()
        self.active.clear()
        self._caps.clear()
        self.used = 0

    def updates_done(self) -> int:
        """Site updates enqueued so far (finished jobs and the resident ones)."""
        return sum(r.updates() for r in self.done) + self._cancelled_updates + sum(
            2 * req.L ** 3 * job.sweeps_done() for job, req, _ in self.active.values())

    def serve(self, requests, clock=time.perf_counter, sleep=time.sleep, cap_s=None):
        """Run a stream of requests (any order; served by arrival) to completion,
        or until cap_s seconds of wall clock (then the in-flight work is waited
        for and the unfinished requests are left without t_done)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = clock()
        i = 0
        while i < len(reqs) or self.pending or self.creating or self.active:
            now = clock() - t0
            if cap_s is not None and now >= cap_s:
                break
            while i < len(reqs) and reqs[i].arrival <= now:
                if reqs[i].rid in self._cancel:
                    self._mark_cancelled(reqs[i])
                else:
                    self.pending.append(reqs[i])
                i += 1
            self._admit()
            while self.inflight and self.be.done(self.inflight[0]):
                self.inflight.popleft()
            finished, ready = self._finished(), self._ready()
            leaving = any(r in self.active for r in self._cancel)
            if finished or ready or leaving:
                # membership changes at a period boundary: let the enqueued
                # periods end, release finished jobs, add the new ones
                ta = clock()
                self._drain()
                tb = clock()
                now = tb - t0
                self._harvest(finished, now)
                self._drop_cancelled()
                self._join(ready, now)
                self._set_caps()
                self._admit()
                self.changes += 1
                self.host_s["drain"] += tb - ta
                self.host_s["change"] += clock() - tb
            if self.active and len(self.inflight) < self.depth:
                ta = clock()
                self._launch()
                self.host_s["launch"] += clock() - ta
            elif self.inflight:
                ta = clock()
                self.be.wait(self.inflight[0])
                self.host_s["wait"] += clock() - ta
            elif i < len(reqs) or self.creating:
                # nothing on the device: wait for the next arrival or for a
                # job being created (never a zero-length sleep, which would
                # keep the interpreter lock from the creating threads)
                nxt = reqs[i].arrival - (clock() - t0) if i < len(reqs) else 0.002
                sleep(max(0.0005, min(0.002, nxt)))
        self._drain()
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


def summary(done, wall: float, updates=None):
    """Latency percentiles of the completed requests and throughput; updates
    (if given) counts all the sweeps performed, finished jobs or not."""
    lat = np.array([r.latency for r in done]) if done else np.zeros(1)
    upd = sum(r.updates() for r in done) if updates is None else updates
    return {"jobs": len(done), "wall_s": round(wall, 3),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "jobs_per_s": round(len(done) / wall, 3),
            "updates_per_ns": round(upd / (wall * 1e9), 3)}
