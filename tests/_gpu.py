"""Helpers shared by the GPU parity tests (run the same seeded inputs through
the oracle and through libsg, compare element by element)."""
import numpy as np

import oracle
from paper_0704_3573_amd import inputs

MODELS = {"ising": oracle.ISING, "potts": oracle.POTTS, "gpotts": oracle.GPOTTS,
          "rfim": oracle.ISING_GEN, "daff": oracle.ISING_GEN, "isinggen": oracle.ISING_GEN,
          "gpotts4": oracle.GPOTTS4}


def instance(model, L, S=1, R=1, K=1, seed=1, sample0=0):
    return inputs.make_instance(model, L, S, R, K, seed, sample0)


def make_job(ctx, model, algo, L, betas, inst, S=1, R=1, pt_every=0, stream=None, field=0.0):
    from paper_0704_3573_amd import binding as B
    return B.Job(ctx, MODELS[model], algo, L, betas, inst["J"], inst["spins"], inst["wheels"],
                 inst["ptwheels"] if pt_every else None, n_samples=S, n_replicas=R,
                 pt_every=pt_every, stream=stream, field=field)


def run_oracle(model, algo, L, betas, inst, S=1, R=1, n=1, pt_every=0, measure_every=0,
               threads=8, sweeps_done=0, state=None, field=0.0):
    st = state or inst
    return oracle.run(MODELS[model], algo, L, betas, inst["J"], st["spins"], st["wheels"],
                      st.get("ptwheels", inst["ptwheels"]), st.get("slot_of_temp"),
                      n_samples=S, n_replicas=R, n_sweeps=n, sweeps_done=sweeps_done,
                      pt_every=pt_every, measure_every=measure_every, n_threads=threads,
                      field=field)


def assert_same_state(job, ref, what=""):
    sp = job.spins()
    assert np.array_equal(sp, ref["spins"]), f"spins differ {what}: " \
        f"{int((sp != ref['spins']).sum())} of {sp.size} sites"
    wh, pw = job.wheels()
    assert np.array_equal(wh, ref["wheels"]), f"wheels differ {what}"
    E = job.energies()
    assert np.array_equal(E, ref["E"]), f"energies differ {what}: {E[:4]} vs {ref['E'][:4]}"
    if job.model == 3:  # Ising-like: field sums by temperature (no PT: slot order)
        M = job.field_sums()
        assert np.array_equal(M, ref["M"]), f"field sums differ {what}: {M[:4]} vs {ref['M'][:4]}"
    if job.K > 1 and job.spec.pt_every:
        assert np.array_equal(job.perm(), ref["slot_of_temp"]), f"PT permutation differs {what}"
        assert np.array_equal(pw, ref["ptwheels"]), f"PT wheels differ {what}"
