"""GPU parity of the glassy Potts model of Eq. (3) on the 4D hypercubic
lattice (the paper's 4D runs): libsg against the CPU oracle on the same
seeded inputs, bit for bit (spins, wheel states, energies, overlaps,
parallel-tempering permutations)."""
import numpy as np
import pytest

import oracle
from paper_0704_3573_amd import inputs
from tests._gpu import assert_same_state, instance, make_job, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0704_3573_amd import binding as B
    return B.Context(0)


@pytest.mark.parametrize("L", [2, 4, 8, 16])
def test_4d_sweeps_match_oracle(ctx, L):
    S, R = (3, 2) if L <= 8 else (1, 2)
    inst = instance("gpotts4", L, S=S, R=R, seed=700 + L)
    job = make_job(ctx, "gpotts4", oracle.HEATBATH, L, [1.405], inst, S=S, R=R)
    n = 3 if L == 16 else 7
    job.sweep(n)
    ref = run_oracle("gpotts4", oracle.HEATBATH, L, [1.405], inst, S=S, R=R, n=n)
    assert_same_state(job, ref, f"4D L={L}")


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.405, 3.0, 60.0])
def test_4d_temperatures(ctx, beta):
    L = 8
    inst = instance("gpotts4", L, S=1, R=2, seed=710)
    job = make_job(ctx, "gpotts4", oracle.HEATBATH, L, [beta], inst, R=2)
    job.sweep(5)
    ref = run_oracle("gpotts4", oracle.HEATBATH, L, [beta], inst, R=2, n=5)
    assert_same_state(job, ref, f"4D beta={beta}")


def test_4d_measurements_and_parallel_tempering(ctx):
    L, S, R, K, pe = 4, 3, 2, 4, 2
    betas = 1.0 / np.linspace(0.5, 1.2, K)
    inst = instance("gpotts4", L, S=S, R=R, K=K, seed=720)
    job = make_job(ctx, "gpotts4", oracle.HEATBATH, L, betas, inst, S=S, R=R, pt_every=pe)
    E_gpu, Q_gpu = [], []
    for _ in range(3):
        job.sweep(4)
        E, Q = job.measure()
        E_gpu.append(E)
        Q_gpu.append(Q)
    ref = run_oracle("gpotts4", oracle.HEATBATH, L, betas, inst, S=S, R=R, n=12, pt_every=pe,
                     measure_every=4)
    assert np.array_equal(np.array(E_gpu), ref["E_log"])
    assert np.array_equal(np.array(Q_gpu), ref["Q_log"].reshape(3, -1))
    assert_same_state(job, ref, "4D PT")


def test_4d_in_a_mixed_batch(ctx):
    from paper_0704_3573_amd import binding as B
    specs = [("gpotts4", oracle.HEATBATH, 16, 1, 2), ("gpotts", oracle.HEATBATH, 16, 1, 2),
             ("gpotts4", oracle.HEATBATH, 4, 2, 2), ("ising", oracle.METROPOLIS, 16, 1, 2),
             ("rfim", oracle.METROPOLIS, 8, 1, 2)]
    jobs = []
    for n, (model, algo, L, S, R) in enumerate(specs):
        inst = instance(model, L, S, R, seed=730 + n)
        beta = 1.0 / (0.5 + 0.2 * n)
        jobs.append((model, algo, L, S, R, beta, inst,
                     make_job(ctx, model, algo, L, [beta], inst, S=S, R=R, field=1.0 if model == "rfim" else 0.0)))
    for block in (512, 1024):
        batch = B.Batch(ctx, [j[-1] for j in jobs], block=block)
        batch.run(2)
        batch.run(1)
        batch.close()
    for model, algo, L, S, R, beta, inst, job in jobs:
        ref = run_oracle(model, algo, L, [beta], inst, S=S, R=R, n=6,
                         field=1.0 if model == "rfim" else 0.0)
        assert_same_state(job, ref, f"mixed batch {model} L={L}")


def test_4d_checkpoint_resume_is_bit_exact(ctx):
    from paper_0704_3573_amd import binding as B
    L, S, R = 8, 1, 2
    inst = instance("gpotts4", L, S, R, seed=740)
    full = make_job(ctx, "gpotts4", oracle.HEATBATH, L, [1.405], inst, S=S, R=R)
    full.sweep(9)
    part = make_job(ctx, "gpotts4", oracle.HEATBATH, L, [1.405], inst, S=S, R=R)
    part.sweep(5)
    wh, _ = part.wheels()
    resumed = B.Job(ctx, B.GPOTTS4, B.HEATBATH, L, [1.405], inst["J"], part.spins(), wh,
                    n_samples=S, n_replicas=R, sweeps_done=5)
    resumed.sweep(4)
    assert np.array_equal(resumed.spins(), full.spins())
    assert np.array_equal(resumed.wheels()[0], full.wheels()[0])
    assert np.array_equal(resumed.measure()[0], full.measure()[0])


def test_4d_paper_workload_sampled_chains(ctx):
    # the paper's 4D runs: L = 16 at beta = 1.405; here 128 samples x 2
    # replicas for 200 sweeps, samples 0 and 99 re-run by the oracle
    L, S, R, n = 16, 128, 2, 200
    inst = instance("gpotts4", L, S=S, R=R, seed=4600)
    job = make_job(ctx, "gpotts4", oracle.HEATBATH, L, [1.405], inst, S=S, R=R)
    for _ in range(4):
        job.sweep(n // 4)
    E, Q = job.measure()
    sp = job.spins()
    for s in (0, 99):
        sub = {"J": inst["J"][s:s + 1], "spins": inst["spins"][2 * s:2 * s + 2],
               "wheels": inst["wheels"][2 * s:2 * s + 2], "ptwheels": inst["ptwheels"][:2]}
        ref = run_oracle("gpotts4", oracle.HEATBATH, L, [1.405], sub, R=R, n=n, measure_every=n,
                         threads=2)
        assert np.array_equal(sp[2 * s:2 * s + 2], ref["spins"])
        assert np.array_equal(E[2 * s:2 * s + 2], ref["E_log"][0].reshape(-1))
        assert Q[s] == ref["Q_log"][0, 0, 0]


def test_4d_invalid_permutation_bytes_are_rejected(ctx):
    from paper_0704_3573_amd import binding as B
    inst = instance("gpotts4", 4, seed=750)
    bad = dict(inst, J=inst["J"].copy())
    bad["J"][0, 3, 7] = 0x00
    with pytest.raises(B.SgError) as e:
        make_job(ctx, "gpotts4", oracle.HEATBATH, 4, [1.0], bad)
    assert e.value.code == B.SG_E_INVALID
