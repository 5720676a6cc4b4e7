"""CPU tests of the serving loop's scheduling: admission by slots and memory
budget, FIFO order, exact per-job sweep counts under continuous batching.
A fake backend counts sweeps instead of launching kernels (its jobs are
created at once and its periods end at once)."""
import pytest

from paper_0704_3573_amd.serving import Request, Server, poisson_stream, summary


class FakeJob:
    def __init__(self, req):
        self.req = req
        self.done = 0
        self.closed = False

    def sweeps_done(self):
        return self.done

    def close(self):
        self.closed = True


class FakeBatch:
    def __init__(self):
        self.jobs = []
        self.budgets = {}
        self.caps = {}
        self.runs = []

    def add(self, j):
        assert j not in self.jobs
        self.jobs.append(j)

    def remove(self, j):
        self.jobs.remove(j)
        self.budgets.pop(id(j))

    def set_budget(self, j, n):
        self.budgets[id(j)] = n

    def set_period_cap(self, j, n):
        self.caps[id(j)] = n

    def run(self, n):
        self.runs.append((n, len(self.jobs)))
        for j in self.jobs:
            k = min(n, self.budgets[id(j)], self.caps.get(id(j), n))
            j.done += k
            self.budgets[id(j)] -= k


class FakeBackend:
    def __init__(self, clock):
        self.clock = clock
        self.created = []

    def new_batch(self):
        return FakeBatch()

    def job_bytes(self, req):
        return req.L ** 3  # stand-in size

    def create_async(self, req):
        self.created.append(req.rid)
        return FakeJob(req)

    @staticmethod
    def ready(handle):
        return True

    @staticmethod
    def take(handle):
        return handle

    def launch(self, batch, n):
        batch.run(n)
        self.clock.t += 1e-6 * n * len(batch.jobs)
        return object()

    @staticmethod
    def done(token):
        return True

    @staticmethod
    def wait(token):
        pass

    def finish(self, job, req):
        assert job.done == req.sweeps
        req.E = [job.done, -job.done]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def run(reqs, budget, slots, period):
    clock = Clock()
    be = FakeBackend(clock)
    srv = Server(be, hbm_budget=budget, max_slots=slots, period=period)
    done = srv.serve(reqs, clock=clock, sleep=clock.sleep)
    return srv, be, done


def test_every_job_runs_exactly_its_sweeps():
    reqs = poisson_stream(60, rate=2000.0, seed=3, sweeps_lo=1.0, sweeps_hi=3.0)
    srv, be, done = run(reqs, budget=10 ** 9, slots=8, period=77)
    assert len(done) == 60
    assert all(r.E == [r.sweeps, -r.sweeps] for r in done)
    assert srv.peak_slots <= 8
    assert all(r.t_admit >= r.arrival and r.t_done >= r.t_admit for r in done)


def test_admission_respects_memory_budget_and_fifo():
    reqs = [Request(i, "ising", L, 1.0, 50, i, arrival=0.0) for i, L in
            enumerate([48, 8, 8, 48, 16, 48, 8])]
    budget = 48 ** 3 + 2 * 8 ** 3
    srv, be, done = run(reqs, budget=budget, slots=100, period=10)
    assert srv.peak_used <= budget
    # FIFO: a large job blocks later small ones until memory frees up
    assert be.created == [0, 1, 2, 3, 4, 5, 6]
    assert len(done) == 7


def test_oversized_request_is_rejected():
    with pytest.raises(RuntimeError):
        run([Request(0, "ising", 48, 1.0, 10, 0)], budget=1000, slots=4, period=10)


def test_jobs_join_while_others_run():
    reqs = [Request(0, "ising", 8, 1.0, 1000, 0, arrival=0.0),
            Request(1, "potts", 8, 1.0, 100, 1, arrival=1e-4)]
    srv, be, done = run(reqs, budget=10 ** 9, slots=4, period=100)
    assert [r.rid for r in done] == [1, 0]
    # the second job joined a batch that already held the first
    assert any(k == 2 for _, k in srv.batch.runs)


def test_summary_percentiles():
    reqs = poisson_stream(30, rate=500.0, seed=4, sweeps_lo=1.0, sweeps_hi=2.0)
    srv, be, done = run(reqs, budget=10 ** 9, slots=16, period=50)
    s = summary(done, wall=1.0)
    assert s["jobs"] == 30 and s["p99_latency_s"] >= s["p50_latency_s"] >= 0


def test_periods_give_every_job_the_same_device_time():
    from paper_0704_3573_amd.serving import sweep_cost
    reqs = [Request(0, "ising", 8, 1.0, 700, 0), Request(1, "ising", 16, 1.0, 2000, 1),
            Request(2, "potts", 48, 1.0, 90, 2)]
    # an L = 48 Potts wheel is served by two lanes
    assert sweep_cost(reqs[2]) == 8 * 48 * 8 / 2 and sweep_cost(reqs[1]) == 2 * sweep_cost(reqs[0])
    srv, be, done = run(reqs, budget=10 ** 9, slots=8, period=30)
    # period 1: the L = 48 Potts job runs 30 sweeps; the L = 16 job 30 * 1536
    # / 128 = 360, the L = 8 one 720, capped at its 700
    assert srv.batch.runs[0] == (700, 3)
    assert [r.rid for r in done][0] == 0
    assert all(r.E == [r.sweeps, -r.sweeps] for r in done) and len(done) == 3
    assert srv.updates_done() == sum(r.updates() for r in done)


def test_wall_clock_cap_stops_with_work_left():
    reqs = [Request(0, "ising", 8, 1.0, 10 ** 6, 0), Request(1, "ising", 8, 1.0, 50, 1)]
    clock = Clock()
    be = FakeBackend(clock)
    srv = Server(be, hbm_budget=10 ** 9, max_slots=4, period=100)
    done = srv.serve(reqs, clock=clock, sleep=clock.sleep, cap_s=0.01)
    assert [r.rid for r in done] == [1] and reqs[0].t_done is None
    assert srv.updates_done() > reqs[1].updates()


def test_release_after_the_cap_closes_every_job():
    reqs = [Request(i, "ising", 8, 1.0, 10 ** 6, i) for i in range(6)]
    clock = Clock()
    be = FakeBackend(clock)
    srv = Server(be, hbm_budget=10 ** 9, max_slots=4, period=100)
    srv.serve(reqs, clock=clock, sleep=clock.sleep, cap_s=0.001)
    held = [job for job, _, _ in srv.active.values()]
    assert held and not srv.done
    srv.release()
    assert all(j.closed for j in held) and not srv.active and not srv.creating
    assert srv.used == 0 and srv.batch.jobs == []


class CancellingBackend(FakeBackend):
    """Cancels requests after given numbers of period launches."""

    def __init__(self, clock, plan):
        super().__init__(clock)
        self.plan = plan          # launches -> rids to cancel then
        self.srv = None
        self.launches = 0

    def launch(self, batch, n):
        tok = super().launch(batch, n)
        self.launches += 1
        for rid in self.plan.get(self.launches, ()):
            self.srv.cancel(rid)
        return tok


def test_cancelled_requests_leave_and_the_others_run_exactly():
    reqs = [Request(0, "ising", 8, 1.0, 10 ** 6, 0, arrival=0.0),     # resident, cancelled
            Request(1, "ising", 16, 1.0, 3000, 1, arrival=0.0),        # runs to completion
            Request(2, "ising", 8, 1.0, 500, 2, arrival=0.0),          # waits for a slot, cancelled
            Request(3, "potts", 8, 1.0, 400, 3, arrival=10.0)]         # cancelled before arrival
    clock = Clock()
    be = CancellingBackend(clock, {3: [0, 2, 3]})
    srv = Server(be, hbm_budget=10 ** 9, max_slots=2, period=50)
    be.srv = srv
    done = srv.serve(reqs, clock=clock, sleep=clock.sleep)
    assert [r.rid for r in done] == [1] and done[0].E == [3000, -3000]
    assert sorted(r.rid for r in srv.cancelled) == [0, 2, 3]
    assert all(r.cancelled and r.t_done is None for r in srv.cancelled)
    assert 2 not in be.created and 3 not in be.created   # never created
    assert srv.used == 0 and not srv.active and srv.batch.jobs == []
    # the cancelled resident job's sweeps count as performed work
    assert srv.updates_done() > done[0].updates()
    assert srv.cancel(1) is False                         # already completed
