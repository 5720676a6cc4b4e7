"""GPU parity of the batched form: jobs of mixed L advanced by one fused
launch per period (hipGraph replay) must reproduce the oracle and their own
stand-alone runs bit for bit, for every block size, and when jobs join or
leave the batch between runs."""
import numpy as np
import pytest

import oracle
from paper_0704_3573_amd import inputs
from tests._gpu import assert_same_state, instance, make_job, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_0704_3573_amd import binding as B
    return B.Context(0)


def small_jobs(ctx, pe=3):
    specs = [("ising", oracle.METROPOLIS, 8, 2, 2, 4), ("ising", oracle.METROPOLIS, 16, 1, 2, 3),
             ("ising", oracle.HEATBATH, 24, 1, 1, 2), ("potts", oracle.HEATBATH, 16, 2, 2, 1),
             ("ising", oracle.METROPOLIS, 48, 1, 2, 2)]
    out = []
    for n, (model, algo, L, S, R, K) in enumerate(specs):
        betas = 1.0 / np.linspace(0.8, 1.5, K)
        inst = instance(model, L, S, R, K, seed=700 + n)
        job = make_job(ctx, model, algo, L, betas, inst, S=S, R=R, pt_every=pe if K > 1 else 0)
        out.append((model, algo, L, S, R, K, betas, inst, job))
    return out


def test_mixed_batch_matches_oracle_and_alone(ctx):
    from paper_0704_3573_amd import binding as B
    pe = 3
    jobs = small_jobs(ctx, pe)
    alone = small_jobs(ctx, pe)
    batch = B.Batch(ctx, [j[-1] for j in jobs])
    batch.run(4)
    batch.run(5)
    for (model, algo, L, S, R, K, betas, inst, job), a in zip(jobs, alone):
        a[-1].sweep(9)
        ref = run_oracle(model, algo, L, betas, inst, S=S, R=R, n=9, pt_every=pe if K > 1 else 0)
        assert_same_state(job, ref, f"batched {model} L={L}")
        assert np.array_equal(job.spins(), a[-1].spins())
        assert np.array_equal(job.wheels()[0], a[-1].wheels()[0])


@pytest.mark.parametrize("block", [64 * k for k in (8, 9, 12, 16)])
def test_batch_block_size_does_not_change_results(ctx, block):
    from paper_0704_3573_amd import binding as B
    jobs = small_jobs(ctx)
    batch = B.Batch(ctx, [j[-1] for j in jobs], block=block)
    assert batch.block() == block
    batch.run(6)
    for model, algo, L, S, R, K, betas, inst, job in jobs:
        ref = run_oracle(model, algo, L, betas, inst, S=S, R=R, n=6, pt_every=3 if K > 1 else 0)
        assert_same_state(job, ref, f"block={block} {model} L={L}")


def test_continuous_batching_join_and_leave(ctx):
    from paper_0704_3573_amd import binding as B
    jobs = small_jobs(ctx)
    batch = B.Batch(ctx, [jobs[0][-1], jobs[1][-1]])
    batch.run(3)
    batch.add(jobs[2][-1])
    batch.add(jobs[3][-1])
    batch.run(4)
    batch.remove(jobs[0][-1])
    batch.add(jobs[4][-1])
    batch.run(2)
    want = [7, 9, 6, 6, 2]
    for (model, algo, L, S, R, K, betas, inst, job), n in zip(jobs, want):
        assert job.sweeps_done() == n
        ref = run_oracle(model, algo, L, betas, inst, S=S, R=R, n=n, pt_every=3 if K > 1 else 0)
        assert_same_state(job, ref, f"continuous {model} L={L}")



def test_fused_and_unfused_parallel_tempering_in_one_batch(ctx):
    """A K = 70 job takes the unfused parallel-tempering kernel and is due
    every sweep; a K = 3 job is due every second sweep, and its fused PT
    launch then also advances every job's sweep counter; in the other
    periods the counters advance in a launch of their own.  A job without PT
    rides along.  Every job must match the oracle."""
    from paper_0704_3573_amd import binding as B
    specs = [("ising", oracle.METROPOLIS, 4, 1, 1, 70, 1), ("ising", oracle.METROPOLIS, 8, 1, 2, 3, 2),
             ("ising", oracle.HEATBATH, 8, 1, 1, 1, 0)]
    jobs = []
    for n, (model, algo, L, S, R, K, pe) in enumerate(specs):
        betas = 1.0 / np.linspace(0.5, 3.0, K) if K > 1 else [1.0 / 1.1]
        inst = instance(model, L, S, R, K, seed=980 + n)
        jobs.append((model, algo, L, S, R, K, pe, betas, inst,
                     make_job(ctx, model, algo, L, betas, inst, S=S, R=R, pt_every=pe)))
    batch = B.Batch(ctx, [j[-1] for j in jobs])
    batch.run(3)
    batch.run(4)
    for model, algo, L, S, R, K, pe, betas, inst, job in jobs:
        assert job.sweeps_done() == 7
        ref = run_oracle(model, algo, L, betas, inst, S=S, R=R, n=7, pt_every=pe)
        assert_same_state(job, ref, f"{model} L={L} K={K}")

def test_full_size_batched_pt_workload_sampled_chains(ctx):
    """The benchmark's batched workload at full size (256 samples at L = 16,
    24, 32, 48, 2 replicas x 32 temperatures, PT every 10 sweeps) in the
    launch configuration the benchmark times; one sample per L (all 64 of its
    copies) is re-run by the oracle."""
    from paper_0704_3573_amd import binding as B
    betas = 1.0 / inputs.linear_temperatures(32, 0.7, 1.6)
    jobs, insts = [], []
    for i, L in enumerate((16, 24, 32, 48)):
        inst = inputs.make_instance("ising", L, 64, 2, 32, seed=3000, sample0=64 * i)
        jobs.append(B.Job(ctx, B.ISING, B.METROPOLIS, L, betas, inst["J"], inst["spins"],
                          inst["wheels"], inst["ptwheels"], n_samples=64, n_replicas=2,
                          pt_every=10))
        # keep the inputs of sample 5 of this job only
        s = 5
        insts.append({"J": inst["J"][s:s + 1].copy(), "spins": inst["spins"][s * 64:(s + 1) * 64].copy(),
                      "wheels": inst["wheels"][s * 64:(s + 1) * 64].copy(),
                      "ptwheels": inst["ptwheels"][s * 2:(s + 1) * 2].copy()})
        del inst
    batch = B.Batch(ctx, jobs)
    assert batch.block() % 64 == 0 and batch.block() >= 288
    batch.run(20)
    for L, job, inst in zip((16, 24, 32, 48), jobs, insts):
        ref = oracle.run(oracle.ISING, oracle.METROPOLIS, L, betas, inst["J"], inst["spins"],
                         inst["wheels"], inst["ptwheels"], n_samples=1, n_replicas=2, n_sweeps=20,
                         pt_every=10, n_threads=8)
        sp = job.spins()[5 * 64:6 * 64]
        assert np.array_equal(sp, ref["spins"]), f"L={L}"
        assert np.array_equal(job.energies()[5 * 64:6 * 64], ref["E"]), f"L={L}"
        assert np.array_equal(job.perm()[10:12], ref["slot_of_temp"]), f"L={L}"
        wh, pw = job.wheels()
        assert np.array_equal(wh[5 * 64:6 * 64], ref["wheels"]), f"L={L}"
        assert np.array_equal(pw[10:12], ref["ptwheels"]), f"L={L}"


@pytest.mark.parametrize("block", [320, 448, 512, 1024])
def test_partial_waves_match_oracle(ctx, block):
    """Copies whose wheel count is not a multiple of 64 (L = 24, 40, 48, and an
    odd number of L = 16 Potts copies) leave lanes without a wheel in a live
    wave; those lanes must not disturb any result, at every block size (the
    Potts launch uses at most 512 threads)."""
    from paper_0704_3573_amd import binding as B
    specs = [("potts", oracle.HEATBATH, 48, 1, 1, 1), ("potts", oracle.HEATBATH, 40, 1, 1, 1),
             ("potts", oracle.HEATBATH, 24, 1, 3, 1), ("potts", oracle.HEATBATH, 16, 1, 3, 1),
             ("ising", oracle.METROPOLIS, 24, 1, 3, 1), ("ising", oracle.HEATBATH, 40, 1, 1, 1)]
    jobs = []
    for n, (model, algo, L, S, R, K) in enumerate(specs):
        betas = [1.0 / (0.8 + 0.1 * n)]
        inst = instance(model, L, S, R, K, seed=900 + n)
        jobs.append((model, algo, L, S, R, betas, inst,
                     make_job(ctx, model, algo, L, betas, inst, S=S, R=R)))
    batch = B.Batch(ctx, [j[-1] for j in jobs], block=block)
    batch.run(3)
    batch.run(2)
    for model, algo, L, S, R, betas, inst, job in jobs:
        ref = run_oracle(model, algo, L, betas, inst, S=S, R=R, n=5)
        assert_same_state(job, ref, f"block={block} {model} L={L} copies={S * R}")
