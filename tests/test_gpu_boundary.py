"""GPU: the boundary calls beyond sweep/measure -- jobs created from a seed
alone, sweep(beta, n), checkpoint -> restore -> sweep (bit-exact resume,
also across jobs and after rollback), and batch membership changes on a
non-blocking stream with no host synchronisation between runs."""
import numpy as np
import pytest

import oracle
from paper_0704_3573_amd import inputs
from tests._gpu import MODELS, assert_same_state, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_0704_3573_amd import binding as B
    return B.Context(0)


def lib_model(name):
    from paper_0704_3573_amd import binding as B
    return {"ising": B.ISING, "potts": B.POTTS, "gpotts": B.GPOTTS, "gpotts4": B.GPOTTS4,
            "isinggen": B.ISING_GEN}[name]


@pytest.mark.parametrize("name,algo,L", [("ising", oracle.METROPOLIS, 16),
                                         ("potts", oracle.HEATBATH, 8),
                                         ("gpotts", oracle.HEATBATH, 8),
                                         ("gpotts4", oracle.HEATBATH, 4),
                                         ("isinggen", oracle.HEATBATH, 8)])
def test_seed_created_job_matches_oracle(ctx, name, algo, L):
    from paper_0704_3573_amd import binding as B
    S, R, K, seed, s0 = 2, 2, 2, 4242, 3
    betas = [0.7, 1.1]
    field = 0.6 if name == "isinggen" else 0.0
    pe = 2 if name in ("ising", "potts") else 0
    job = B.Job(ctx, lib_model(name), algo, L, betas, n_samples=S, n_replicas=R, pt_every=pe,
                field=field, seed=seed, sample0=s0)
    job.sweep(5)
    inst = inputs.make_instance(name, L, S, R, K, seed, s0)
    ref = oracle.run(MODELS[name], algo, L, betas, inst["J"], inst["spins"], inst["wheels"],
                     inst["ptwheels"], n_samples=S, n_replicas=R, n_sweeps=5, pt_every=pe,
                     n_threads=4, field=field)
    assert_same_state(job, ref, f"seed-created {name} L={L}")


def test_sweep_beta_equals_set_betas_then_sweep(ctx):
    from paper_0704_3573_amd import binding as B
    L = 16
    a = B.Job(ctx, B.ISING, B.METROPOLIS, L, [1.0], n_replicas=2, seed=77)
    b = B.Job(ctx, B.ISING, B.METROPOLIS, L, [1.0], n_replicas=2, seed=77)
    schedule = [(1.0, 3), (0.5, 4), (0.5, 2), (1 / 0.8, 5)]
    for beta, n in schedule:
        a.sweep_beta(beta, n)
        b.set_betas([beta])
        b.sweep(n)
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.wheels()[0], b.wheels()[0])
    # and against the oracle, piece by piece
    inst = inputs.make_instance("ising", L, 1, 2, 1, 77)
    state = None
    for beta, n in schedule:
        state = run_oracle("ising", oracle.METROPOLIS, L, [beta], inst, R=2, n=n, state=state)
    assert np.array_equal(a.spins(), state["spins"])
    with pytest.raises(B.SgError):
        B.Job(ctx, B.ISING, B.METROPOLIS, L, [1.0, 0.5], seed=1).sweep_beta(1.0, 1)


@pytest.mark.parametrize("name,algo,L,pe", [("ising", oracle.METROPOLIS, 24, 3),
                                            ("potts", oracle.HEATBATH, 16, 2),
                                            ("isinggen", oracle.METROPOLIS, 8, 0)])
def test_checkpoint_restore_is_bit_exact(ctx, name, algo, L, pe):
    from paper_0704_3573_amd import binding as B
    S, R, K = 2, 2, 3
    # close temperatures, so that swaps are accepted within a few steps
    betas = 1.0 / np.linspace(1.0, 1.02, K)
    kw = dict(n_samples=S, n_replicas=R, pt_every=pe, seed=515,
              field=0.4 if name == "isinggen" else 0.0)
    full = B.Job(ctx, lib_model(name), algo, L, betas, **kw)
    full.sweep(13)
    part = B.Job(ctx, lib_model(name), algo, L, betas, **kw)
    part.sweep(7)
    blob = part.checkpoint()
    # restore into a fresh job of the same instance and continue
    other = B.Job(ctx, lib_model(name), algo, L, betas, **kw)
    other.restore(blob)
    assert other.sweeps_done() == 7
    other.sweep(6)
    # rollback: the checkpointed job runs on, is restored and runs again
    part.sweep(4)
    part.restore(blob)
    part.sweep(6)
    for j in (other, part):
        assert np.array_equal(j.spins(), full.spins())
        wa, pa = j.wheels()
        wb, pb = full.wheels()
        assert np.array_equal(wa, wb) and np.array_equal(pa, pb)
        assert np.array_equal(j.perm(), full.perm())
        assert np.array_equal(j.pt_accepts(), full.pt_accepts())
        assert np.array_equal(j.measure()[0], full.measure()[0])
    if pe:
        assert full.pt_accepts().sum() > 0


def test_restore_rejects_other_jobs(ctx):
    from paper_0704_3573_amd import binding as B
    a = B.Job(ctx, B.ISING, B.METROPOLIS, 8, [1.0], seed=1)
    blob = a.checkpoint()
    with pytest.raises(B.SgError) as e:  # other couplings
        B.Job(ctx, B.ISING, B.METROPOLIS, 8, [1.0], seed=2).restore(blob)
    assert e.value.code == B.SG_E_STATE
    with pytest.raises(B.SgError) as e:  # other specification
        B.Job(ctx, B.ISING, B.METROPOLIS, 16, [1.0], seed=1).restore(blob)
    assert e.value.code == B.SG_E_STATE
    with pytest.raises(B.SgError) as e:
        a.restore(b"\0" * len(blob))
    assert e.value.code == B.SG_E_INVALID


def test_arena_one_byte_short_is_rejected(ctx):
    import torch
    from paper_0704_3573_amd import binding as B
    spec = B.Spec(B.ISING, B.METROPOLIS, 4, 16, 1, 2, 1, 0)
    n = B.job_bytes(spec)
    arena = torch.empty(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.SgError) as e:
        B.Job(ctx, B.ISING, B.METROPOLIS, 16, [1.0], n_replicas=2, seed=1, arena=arena[:n - 1])
    assert e.value.code == B.SG_E_NOMEM


def test_membership_changes_on_a_nonblocking_stream_without_host_sync(ctx):
    """Runs, adds and removes are enqueued back to back on a non-blocking
    stream; re-planning must wait for the periods still reading the launch
    tables.  Every job ends where the oracle puts it."""
    import torch
    from paper_0704_3573_amd import binding as B
    specs = [("ising", oracle.METROPOLIS, 16, 1, 2, 3, 2), ("ising", oracle.METROPOLIS, 32, 1, 2, 2, 0),
             ("potts", oracle.HEATBATH, 16, 2, 2, 1, 0), ("ising", oracle.HEATBATH, 24, 1, 2, 1, 0)]
    st = torch.cuda.Stream()
    jobs = []
    for n, (name, algo, L, S, R, K, pe) in enumerate(specs):
        betas = 1.0 / np.linspace(0.8, 1.3, K)
        jobs.append((name, algo, L, S, R, K, pe, betas,
                     B.Job(ctx, lib_model(name), algo, L, betas, n_samples=S, n_replicas=R,
                           pt_every=pe, seed=60 + n, stream=st)))
    batch = B.Batch(ctx, [j[-1] for j in jobs[:2]])
    batch.run(40, st)
    batch.add(jobs[2][-1])
    batch.run(30, st)
    batch.remove(jobs[0][-1])
    batch.add(jobs[3][-1])
    batch.run(20, st)
    batch.remove(jobs[1][-1])
    batch.run(10, st)
    st.synchronize()
    want = [70, 90, 60, 30]
    for k, ((name, algo, L, S, R, K, pe, betas, job), n) in enumerate(zip(jobs, want)):
        assert job.sweeps_done() == n
        inst = inputs.make_instance(name, L, S, R, K, 60 + k)
        ref = run_oracle(name, algo, L, betas, inst, S=S, R=R, n=n, pt_every=pe)
        assert_same_state(job, ref, f"{name} L={L}")


def test_injected_device_errors_leave_jobs_and_batches_intact(ctx, monkeypatch):
    """A device error reported at entry (test hook) changes no state: the
    job's sweep counter, budgets and trajectory continue as if the failing
    calls had not been made."""
    from paper_0704_3573_amd import binding as B
    L, seed = 16, 91
    job = B.Job(ctx, B.ISING, B.METROPOLIS, L, [1.0], n_replicas=2, seed=seed)
    job.sweep(5)
    batch = B.Batch(ctx, [job])
    for fn, call in (("sg_job_sweep", lambda: job.sweep(5)), ("sg_batch_run", lambda: batch.run(4)),
                     ("sg_batch_run_static", lambda: batch.run_static(4)),
                     ("sg_job_measure", lambda: job.measure())):
        monkeypatch.setenv("SG_TEST_INJECT_HIP_ERROR", fn)
        with pytest.raises(B.SgError) as e:
            call()
        assert e.value.code == B.SG_E_HIP, fn
        assert job.sweeps_done() == 5, fn
    monkeypatch.delenv("SG_TEST_INJECT_HIP_ERROR")
    batch.run(4)
    job.sweep(3)
    assert job.sweeps_done() == 12
    inst = inputs.make_instance("ising", L, 1, 2, 1, seed)
    ref = run_oracle("ising", oracle.METROPOLIS, L, [1.0], inst, R=2, n=12)
    assert np.array_equal(job.spins(), ref["spins"])
    assert np.array_equal(job.wheels()[0], ref["wheels"])


def test_results_do_not_depend_on_the_arena_offset(ctx):
    """A job placed at a 256-byte aligned offset inside a larger buffer
    runs exactly as one in an arena of its own; a misaligned arena is
    rejected."""
    import torch
    from paper_0704_3573_amd import binding as B
    L, seed = 16, 333
    spec = B.Spec(B.POTTS, B.HEATBATH, 4, L, 1, 2, 1, 0)
    n = B.job_bytes(spec)
    big = torch.empty(n + 8192, dtype=torch.uint8, device="cuda")
    kw = dict(n_replicas=2, seed=seed)
    a = B.Job(ctx, B.POTTS, B.HEATBATH, L, [1.1], **kw)
    b = B.Job(ctx, B.POTTS, B.HEATBATH, L, [1.1], arena=big[4096 + 256:4096 + 256 + n], **kw)
    for j in (a, b):
        j.sweep(7)
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.wheels()[0], b.wheels()[0])
    assert np.array_equal(a.measure()[0], b.measure()[0])
    with pytest.raises(B.SgError) as e:
        B.Job(ctx, B.POTTS, B.HEATBATH, L, [1.1], arena=big[128:128 + n], **kw)
    assert e.value.code == B.SG_E_INVALID
