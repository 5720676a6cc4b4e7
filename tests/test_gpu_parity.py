"""GPU parity: libsg (HIP, gfx950) against the CPU oracle on the same seeded
inputs.  Spins, wheel states, energies, overlaps and parallel-tempering
permutations must agree bit for bit (every quantity is an integer)."""
import numpy as np
import pytest

import oracle
from tests._gpu import assert_same_state, instance, make_job, run_oracle

pytestmark = pytest.mark.gpu

ISING_L = [2, 4, 8, 16, 24, 32, 40, 48, 56, 64]
POTTS_L = [2, 4, 8, 16, 24, 32, 40, 48]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0704_3573_amd import binding as B
    return B.Context(0)


def test_debug_rng_matches_oracle_stream(ctx):
    inst = instance("ising", 16, seed=41)
    job = make_job(ctx, "ising", oracle.METROPOLIS, 16, [0.9], inst)
    for w in (0, 5, 31):
        got = job.debug_rng(0, w, 1000)
        assert np.array_equal(got, oracle.pr_stream(inst["wheels"][0, w], 1000))
    job.sweep(3)
    wh, _ = job.wheels()
    got = job.debug_rng(0, 7, 500)
    assert np.array_equal(got, oracle.pr_stream(wh[0, 7], 500))
    per = 8 * 16
    assert np.array_equal(got, oracle.pr_stream(inst["wheels"][0, 7], 3 * per + 500)[3 * per:])


@pytest.mark.parametrize("L", ISING_L)
@pytest.mark.parametrize("algo", [oracle.METROPOLIS, oracle.HEATBATH])
def test_ising_sweeps_match_oracle(ctx, L, algo):
    S, K = 2, 2
    betas = [1 / 1.1, 1 / 0.8]
    inst = instance("ising", L, S=S, K=K, seed=100 + L)
    job = make_job(ctx, "ising", algo, L, betas, inst, S=S)
    n = 3 if L >= 48 else 5
    job.sweep(n)
    ref = run_oracle("ising", algo, L, betas, inst, S=S, n=n)
    assert_same_state(job, ref, f"L={L} algo={algo}")


@pytest.mark.parametrize("L", POTTS_L)
def test_potts_sweeps_match_oracle(ctx, L):
    S, R = 2, 2
    betas = [1 / 0.9]
    inst = instance("potts", L, S=S, R=R, seed=200 + L)
    job = make_job(ctx, "potts", oracle.HEATBATH, L, betas, inst, S=S, R=R)
    n = 2 if L >= 40 else 4
    job.sweep(n)
    ref = run_oracle("potts", oracle.HEATBATH, L, betas, inst, S=S, R=R, n=n)
    assert_same_state(job, ref, f"Potts L={L}")


@pytest.mark.parametrize("beta", [0.0, 0.05, 3.0, 60.0])
@pytest.mark.parametrize("algo", [oracle.METROPOLIS, oracle.HEATBATH])
def test_extreme_temperatures(ctx, beta, algo):
    # beta = 0 gives thresholds equal to 2^32 ("always"), beta = 60 gives 0
    L = 16
    inst = instance("ising", L, S=1, K=1, seed=300)
    job = make_job(ctx, "ising", algo, L, [beta], inst)
    job.sweep(4)
    ref = run_oracle("ising", algo, L, [beta], inst, n=4)
    assert_same_state(job, ref, f"beta={beta}")
    if algo == oracle.METROPOLIS and beta == 0.0:
        assert np.array_equal(job.spins()[0], inst["spins"][0])  # four flips


def test_potts_extreme_temperatures(ctx):
    for beta in (0.0, 50.0):
        inst = instance("potts", 8, seed=301)
        job = make_job(ctx, "potts", oracle.HEATBATH, 8, [beta], inst)
        job.sweep(3)
        ref = run_oracle("potts", oracle.HEATBATH, 8, [beta], inst, n=3)
        assert_same_state(job, ref, f"Potts beta={beta}")


def test_many_copies_per_workgroup_mixed_temperatures(ctx):
    # L = 16: 32 lanes per copy, several copies share a workgroup with different
    # temperatures (per-lane thresholds)
    L, S, R, K = 16, 3, 2, 5
    betas = np.linspace(0.5, 1.5, K)
    inst = instance("ising", L, S=S, R=R, K=K, seed=400)
    job = make_job(ctx, "ising", oracle.METROPOLIS, L, betas, inst, S=S, R=R)
    job.sweep(6)
    ref = run_oracle("ising", oracle.METROPOLIS, L, betas, inst, S=S, R=R, n=6)
    assert_same_state(job, ref)
    E, Q = job.measure()
    ref2 = run_oracle("ising", oracle.METROPOLIS, L, betas, inst, S=S, R=R, n=6, measure_every=6)
    assert np.array_equal(E, ref2["E_log"][0].reshape(-1))
    assert np.array_equal(Q, ref2["Q_log"][0].reshape(-1))


def test_sweeps_split_across_calls_equal_one_call(ctx):
    L = 24
    inst = instance("ising", L, S=1, K=1, seed=500)
    a = make_job(ctx, "ising", oracle.METROPOLIS, L, [1.0], inst)
    b = make_job(ctx, "ising", oracle.METROPOLIS, L, [1.0], inst)
    a.sweep(7)
    for n in (1, 2, 1, 3):
        b.sweep(n)
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.wheels()[0], b.wheels()[0])
    ref = run_oracle("ising", oracle.METROPOLIS, L, [1.0], inst, n=7)
    assert_same_state(b, ref)


def test_parallel_tempering_matches_oracle(ctx):
    L, S, R, K, pe = 8, 2, 2, 6, 2
    betas = 1.0 / np.linspace(0.7, 1.6, K)
    inst = instance("ising", L, S=S, R=R, K=K, seed=600)
    job = make_job(ctx, "ising", oracle.METROPOLIS, L, betas, inst, S=S, R=R, pt_every=pe)
    job.sweep(20)
    ref = run_oracle("ising", oracle.METROPOLIS, L, betas, inst, S=S, R=R, n=20, pt_every=pe)
    assert_same_state(job, ref, "PT")
    assert np.array_equal(job.pt_accepts(), ref["pt_accepts"])
    assert ref["pt_accepts"].sum() > 0
    E, Q = job.measure()
    ref2 = run_oracle("ising", oracle.METROPOLIS, L, betas, inst, S=S, R=R, n=20, pt_every=pe,
                      measure_every=20)
    assert np.array_equal(E, ref2["E_log"][0].reshape(-1))
    assert np.array_equal(Q, ref2["Q_log"][0].reshape(-1))


def test_c1_full_run_with_measurements(ctx):
    # 3D EA, L = 8, one sample, T = 1.1, 1000 Metropolis sweeps, E every 100
    L = 8
    inst = instance("ising", L, seed=1)
    job = make_job(ctx, "ising", oracle.METROPOLIS, L, [1 / 1.1], inst)
    Es = []
    for _ in range(10):
        job.sweep(100)
        Es.append(job.measure()[0][0])
    ref = run_oracle("ising", oracle.METROPOLIS, L, [1 / 1.1], inst, n=1000, measure_every=100)
    assert np.array_equal(np.array(Es), ref["E_log"][:, 0])
    assert_same_state(job, ref, "C1")


def test_c2_size_prefix_with_measurements(ctx):
    # L = 64, two replicas sharing couplings, T = 1.1, E and Q every 100 sweeps
    L = 64
    inst = instance("ising", L, R=2, seed=2)
    job = make_job(ctx, "ising", oracle.METROPOLIS, L, [1 / 1.1], inst, R=2)
    Es, Qs = [], []
    for _ in range(2):
        job.sweep(100)
        E, Q = job.measure()
        Es.append(E)
        Qs.append(Q)
    ref = run_oracle("ising", oracle.METROPOLIS, L, [1 / 1.1], inst, R=2, n=200, measure_every=100)
    assert np.array_equal(np.array(Es), ref["E_log"].reshape(2, -1))
    assert np.array_equal(np.array(Qs), ref["Q_log"].reshape(2, -1))
    assert_same_state(job, ref, "C2")


@pytest.mark.parametrize("model,algo,L", [("ising", oracle.METROPOLIS, 24),
                                          ("ising", oracle.HEATBATH, 16),
                                          ("potts", oracle.HEATBATH, 16)])
def test_checkpoint_resume_is_bit_exact(ctx, model, algo, L):
    from paper_0704_3573_amd import binding as B
    S, R, K, pe = 1, 2, 3, (2 if model == "ising" else 0)
    betas = 1.0 / np.linspace(0.8, 1.4, K)
    inst = instance(model, L, S, R, K, seed=950)
    full = make_job(ctx, model, algo, L, betas, inst, S=S, R=R, pt_every=pe)
    full.sweep(9)
    part = make_job(ctx, model, algo, L, betas, inst, S=S, R=R, pt_every=pe)
    part.sweep(5)
    wh, pw = part.wheels()
    resumed = B.Job(ctx, B.ISING if model == "ising" else B.POTTS, algo, L, betas, inst["J"],
                    part.spins(), wh, pw if pe else None, n_samples=S, n_replicas=R, pt_every=pe,
                    slot_of_temp=part.perm(), sweeps_done=5)
    resumed.sweep(4)
    assert np.array_equal(resumed.spins(), full.spins())
    assert np.array_equal(resumed.wheels()[0], full.wheels()[0])
    assert np.array_equal(resumed.perm(), full.perm())
    assert np.array_equal(resumed.measure()[0], full.measure()[0])


def test_parallel_tempering_many_temperatures(ctx):
    # K > 64 takes the unfused parallel-tempering kernel
    L, S, R, K, pe = 4, 1, 1, 70, 1
    betas = 1.0 / np.linspace(0.5, 3.0, K)
    inst = instance("ising", L, S=S, R=R, K=K, seed=960)
    job = make_job(ctx, "ising", oracle.METROPOLIS, L, betas, inst, S=S, R=R, pt_every=pe)
    job.sweep(6)
    ref = run_oracle("ising", oracle.METROPOLIS, L, betas, inst, S=S, R=R, n=6, pt_every=pe)
    assert_same_state(job, ref, "K=70")


def test_potts_c4_shape_sampled_chains_full_length(ctx):
    # q = 4 +-J Potts, L = 16, 128 samples x 2 replicas, heat bath T = 0.9,
    # 10^4 sweeps; samples 0 and 77 re-run by the oracle
    L, S, R = 16, 128, 2
    inst = instance("potts", L, S=S, R=R, seed=4000)
    job = make_job(ctx, "potts", oracle.HEATBATH, L, [1 / 0.9], inst, S=S, R=R)
    for _ in range(10):
        job.sweep(1000)
    E, Q = job.measure()
    sp = job.spins()
    for s in (0, 77):
        sub = {"J": inst["J"][s:s + 1], "spins": inst["spins"][2 * s:2 * s + 2],
               "wheels": inst["wheels"][2 * s:2 * s + 2], "ptwheels": inst["ptwheels"][:2]}
        ref = run_oracle("potts", oracle.HEATBATH, L, [1 / 0.9], sub, R=R, n=10_000,
                         measure_every=10_000, threads=2)
        assert np.array_equal(sp[2 * s:2 * s + 2], ref["spins"])
        assert np.array_equal(E[2 * s:2 * s + 2], ref["E_log"][0].reshape(-1))
        assert Q[s] == ref["Q_log"][0, 0, 0]
