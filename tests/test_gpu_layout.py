"""Device layouts against the canonical arrays (GPU).

* Round trip: a job created from canonical spins and wheel states hands back
  exactly the same arrays before any sweep, for every model and supported L.
  This pins the host packing into the device layouts: the Ising plane strings
  cut into 32-bit block words (rows straddle words at L = 24, 40, 48, 56), the
  wheel slots of the register ring, the Potts byte layouts.
* beta = 0 Metropolis on the EA glass: every move is accepted, so one sweep
  flips every site exactly once (the spins come back negated) and a second
  sweep restores them, whatever the random numbers; the block words of a
  sweep therefore cover every site of both colours exactly once.
"""
import numpy as np
import pytest

import oracle
from _gpu import instance, make_job

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0704_3573_amd import binding as B
    return B.Context(0)


ISING_L = [2, 4, 8, 16, 24, 32, 40, 48, 56, 64]
POTTS_L = [2, 4, 8, 16, 24, 32, 40, 48]
CASES = ([("ising", L) for L in ISING_L] + [("isinggen", L) for L in ISING_L]
         + [("potts", L) for L in POTTS_L] + [("gpotts", L) for L in POTTS_L]
         + [("gpotts4", L) for L in (2, 4, 8, 16)])


@pytest.mark.parametrize("model,L", CASES)
def test_job_returns_its_inputs_before_any_sweep(ctx, model, L):
    algo = oracle.METROPOLIS if model in ("ising", "isinggen") else oracle.HEATBATH
    S, K = 2, 2
    inst = instance(model, L, S=S, K=K, seed=500 + L)
    job = make_job(ctx, model, algo, L, [1.0, 0.8], inst, S=S,
                   field=0.5 if model == "isinggen" else 0.0)
    assert np.array_equal(job.spins(), inst["spins"]), f"{model} L={L}: spins"
    wh, _ = job.wheels()
    assert np.array_equal(wh, inst["wheels"]), f"{model} L={L}: wheels"


@pytest.mark.parametrize("L", ISING_L)
def test_beta_zero_metropolis_flips_every_site_once_per_sweep(ctx, L):
    inst = instance("ising", L, S=1, K=2, seed=600 + L)
    job = make_job(ctx, "ising", oracle.METROPOLIS, L, [0.0, 0.0], inst)
    job.sweep(1)
    assert np.array_equal(job.spins(), -inst["spins"]), f"L={L}: one sweep"
    job.sweep(1)
    assert np.array_equal(job.spins(), inst["spins"]), f"L={L}: two sweeps"
