"""GPU parity of the glassy (permutation) Potts model, Eq. (3): libsg against
the CPU oracle on the same seeded inputs, bit for bit (spins, wheel states,
energies, overlaps, parallel-tempering permutations)."""
import numpy as np
import pytest

import oracle
from paper_0704_3573_amd import inputs
from tests._gpu import assert_same_state, instance, make_job, run_oracle

pytestmark = pytest.mark.gpu

GLASSY_L = [2, 4, 8, 16, 24, 32, 40, 48]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0704_3573_amd import binding as B
    return B.Context(0)


@pytest.mark.parametrize("L", GLASSY_L)
def test_glassy_sweeps_match_oracle(ctx, L):
    S, R = (2, 2) if L <= 32 else (1, 2)
    betas = [2.4]
    inst = instance("gpotts", L, S=S, R=R, seed=300 + L)
    job = make_job(ctx, "gpotts", oracle.HEATBATH, L, betas, inst, S=S, R=R)
    n = 2 if L >= 40 else 5
    job.sweep(n)
    ref = run_oracle("gpotts", oracle.HEATBATH, L, betas, inst, S=S, R=R, n=n)
    assert_same_state(job, ref, f"glassy L={L}")


@pytest.mark.parametrize("beta", [0.0, 0.3, 1.405, 2.4, 60.0])
def test_glassy_temperatures(ctx, beta):
    L = 8
    inst = instance("gpotts", L, S=1, R=2, seed=310)
    job = make_job(ctx, "gpotts", oracle.HEATBATH, L, [beta], inst, R=2)
    job.sweep(7)
    ref = run_oracle("gpotts", oracle.HEATBATH, L, [beta], inst, R=2, n=7)
    assert_same_state(job, ref, f"glassy beta={beta}")


def test_identity_couplings_equal_ferromagnetic_potts_on_gpu(ctx):
    L = 16
    inst = instance("gpotts", L, S=1, R=2, seed=320)
    ident = dict(inst, J=np.full_like(inst["J"], inputs.permutation_bytes()[0]))
    ferro = dict(inst, J=np.ones(inst["J"].shape, np.int8))
    a = make_job(ctx, "gpotts", oracle.HEATBATH, L, [1.3], ident, R=2)
    b = make_job(ctx, "potts", oracle.HEATBATH, L, [1.3], ferro, R=2)
    a.sweep(6)
    b.sweep(6)
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.energies(), b.energies())


def test_glassy_measurements_and_parallel_tempering(ctx):
    L, S, R, K, pe = 8, 2, 2, 4, 2
    betas = 1.0 / np.linspace(0.4, 1.0, K)
    inst = instance("gpotts", L, S=S, R=R, K=K, seed=330)
    job = make_job(ctx, "gpotts", oracle.HEATBATH, L, betas, inst, S=S, R=R, pt_every=pe)
    E_gpu, Q_gpu = [], []
    for _ in range(3):
        job.sweep(4)
        E, Q = job.measure()
        E_gpu.append(E)
        Q_gpu.append(Q)
    ref = run_oracle("gpotts", oracle.HEATBATH, L, betas, inst, S=S, R=R, n=12, pt_every=pe,
                     measure_every=4)
    assert np.array_equal(np.array(E_gpu), ref["E_log"])
    assert np.array_equal(np.array(Q_gpu), ref["Q_log"].reshape(3, -1))
    assert_same_state(job, ref, "glassy PT")


def test_glassy_in_a_mixed_batch(ctx):
    from paper_0704_3573_amd import binding as B
    specs = [("gpotts", oracle.HEATBATH, 16, 1, 3), ("potts", oracle.HEATBATH, 8, 1, 2),
             ("ising", oracle.METROPOLIS, 24, 1, 2), ("gpotts", oracle.HEATBATH, 48, 1, 1)]
    jobs = []
    for n, (model, algo, L, S, R) in enumerate(specs):
        inst = instance(model, L, S, R, seed=340 + n)
        jobs.append((model, algo, L, S, R, inst,
                     make_job(ctx, model, algo, L, [1.0 / (0.5 + 0.2 * n)], inst, S=S, R=R)))
    for block in (320, 1024):
        batch = B.Batch(ctx, [j[-1] for j in jobs], block=block)
        batch.run(2)
        batch.run(1)
        batch.close()
    for model, algo, L, S, R, inst, job in jobs:
        ref = run_oracle(model, algo, L, [1.0 / (0.5 + 0.2 * specs.index((model, algo, L, S, R)))],
                         inst, S=S, R=R, n=6)
        assert_same_state(job, ref, f"mixed batch {model} L={L}")


def test_glassy_checkpoint_resume_is_bit_exact(ctx):
    from paper_0704_3573_amd import binding as B
    L, S, R = 16, 1, 2
    inst = instance("gpotts", L, S, R, seed=350)
    full = make_job(ctx, "gpotts", oracle.HEATBATH, L, [2.4], inst, S=S, R=R)
    full.sweep(9)
    part = make_job(ctx, "gpotts", oracle.HEATBATH, L, [2.4], inst, S=S, R=R)
    part.sweep(5)
    wh, _ = part.wheels()
    resumed = B.Job(ctx, B.GPOTTS, B.HEATBATH, L, [2.4], inst["J"], part.spins(), wh,
                    n_samples=S, n_replicas=R, sweeps_done=5)
    resumed.sweep(4)
    assert np.array_equal(resumed.spins(), full.spins())
    assert np.array_equal(resumed.wheels()[0], full.wheels()[0])
    assert np.array_equal(resumed.measure()[0], full.measure()[0])


def test_glassy_paper_workload_sampled_chains(ctx):
    # the paper's 3D glassy Potts runs: L = 16 at beta = 2.4; here 128 samples
    # x 2 replicas for 2000 sweeps, samples 0 and 101 re-run by the oracle
    L, S, R, n = 16, 128, 2, 2000
    inst = instance("gpotts", L, S=S, R=R, seed=4100)
    job = make_job(ctx, "gpotts", oracle.HEATBATH, L, [2.4], inst, S=S, R=R)
    for _ in range(4):
        job.sweep(n // 4)
    E, Q = job.measure()
    sp = job.spins()
    for s in (0, 101):
        sub = {"J": inst["J"][s:s + 1], "spins": inst["spins"][2 * s:2 * s + 2],
               "wheels": inst["wheels"][2 * s:2 * s + 2], "ptwheels": inst["ptwheels"][:2]}
        ref = run_oracle("gpotts", oracle.HEATBATH, L, [2.4], sub, R=R, n=n, measure_every=n,
                         threads=2)
        assert np.array_equal(sp[2 * s:2 * s + 2], ref["spins"])
        assert np.array_equal(E[2 * s:2 * s + 2], ref["E_log"][0].reshape(-1))
        assert Q[s] == ref["Q_log"][0, 0, 0]


def test_invalid_permutation_bytes_are_rejected(ctx):
    from paper_0704_3573_amd import binding as B
    inst = instance("gpotts", 4, seed=360)
    bad = dict(inst, J=inst["J"].copy())
    bad["J"][0, 1, 5] = 0x00  # all images 0: not a permutation
    with pytest.raises(B.SgError) as e:
        make_job(ctx, "gpotts", oracle.HEATBATH, 4, [1.0], bad)
    assert e.value.code == B.SG_E_INVALID
