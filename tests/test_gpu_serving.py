"""GPU: the continuous-batching server returns, for every request, exactly
what the same job gives when run alone (and what the oracle gives)."""
import numpy as np
import pytest

import oracle
from paper_0704_3573_amd import inputs, serving
from tests._gpu import run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_0704_3573_amd import binding as B
    return B.Context(0)


def test_batch_budgets_stop_jobs_exactly(ctx):
    from paper_0704_3573_amd import binding as B
    from tests._gpu import instance, make_job
    ia = instance("ising", 16, R=2, seed=901)
    ib = instance("potts", 8, R=2, seed=902)
    a = make_job(ctx, "ising", oracle.METROPOLIS, 16, [0.9], ia, R=2)
    b = make_job(ctx, "potts", oracle.HEATBATH, 8, [1.2], ib, R=2)
    batch = B.Batch(ctx, [a, b])
    batch.set_budget(a, 7)
    batch.run(4)
    batch.run(5)
    assert a.sweeps_done() == 7 and b.sweeps_done() == 9 and batch.budget(a) == 0
    ra = run_oracle("ising", oracle.METROPOLIS, 16, [0.9], ia, R=2, n=7)
    rb = run_oracle("potts", oracle.HEATBATH, 8, [1.2], ib, R=2, n=9)
    assert np.array_equal(a.spins(), ra["spins"]) and np.array_equal(b.spins(), rb["spins"])
    assert np.array_equal(a.wheels()[0], ra["wheels"])


def test_served_results_equal_alone_and_oracle(ctx):
    reqs = serving.poisson_stream(16, rate=400.0, seed=11, sweeps_lo=1.3, sweeps_hi=2.4,
                                  sizes=(8, 16, 24))
    srv = serving.Server(serving.DeviceBackend(ctx), hbm_budget=8 << 20, max_slots=5, period=29)
    done = srv.serve(reqs)
    assert len(done) == 16 and 2 <= srv.peak_slots <= 5
    assert srv.periods > len(done) // 5
    # continuous batching: some request was admitted while another was running
    assert any(a.t_admit < b.t_admit < a.t_done for a in done for b in done)
    for r in done:
        alone = serving.Request(r.rid, r.model, r.L, r.T, r.sweeps, r.seed)
        job = serving.make_job(ctx, alone)
        job.sweep(r.sweeps)
        serving.finish(job, alone)
        assert np.array_equal(alone.E, r.E) and alone.Q == r.Q, r
        assert alone.spins_hash == r.spins_hash, r
    for r in done[:3]:
        inst = inputs.make_instance(r.model, r.L, 1, 2, 1, r.seed)
        algo = oracle.METROPOLIS if r.model == "ising" else oracle.HEATBATH
        ref = run_oracle(r.model, algo, r.L, [1.0 / r.T], inst, R=2, n=r.sweeps, measure_every=r.sweeps)
        assert np.array_equal(ref["E_log"][0].reshape(-1), r.E)
        assert int(ref["Q_log"][0, 0, 0]) == r.Q
        assert serving.spins_fingerprint(ref["spins"]) == r.spins_hash


def test_cancelling_resident_jobs_leaves_the_others_exact(ctx):
    """Two resident jobs are cancelled mid-run; every other request still
    ends exactly where it ends alone, and the cancelled jobs' memory and
    slots are released."""

    class Cancelling(serving.DeviceBackend):
        def __init__(self, ctx):
            super().__init__(ctx)
            self.srv, self.n = None, 0

        def launch(self, batch, n):
            tok = super().launch(batch, n)
            self.n += 1
            if self.n == 3:
                for rid in (0, 1):
                    self.srv.cancel(rid)
            return tok

    reqs = serving.poisson_stream(8, rate=0.0, seed=13, sweeps_lo=1.5, sweeps_hi=2.2, sizes=(8, 16))
    reqs[0].sweeps = reqs[1].sweeps = 100000    # still running when cancelled
    be = Cancelling(ctx)
    srv = serving.Server(be, hbm_budget=8 << 20, max_slots=8, period=20)
    be.srv = srv
    done = srv.serve(reqs)
    be.close()
    assert sorted(r.rid for r in srv.cancelled) == [0, 1] and len(done) == 6
    assert srv.used == 0 and not srv.active
    for r in done:
        alone = serving.Request(r.rid, r.model, r.L, r.T, r.sweeps, r.seed)
        job = serving.make_job(ctx, alone)
        job.sweep(r.sweeps)
        serving.finish(job, alone)
        assert np.array_equal(alone.E, r.E) and alone.Q == r.Q and alone.spins_hash == r.spins_hash, r
