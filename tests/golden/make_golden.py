"""Write the full-length parity fixtures of tests/golden/ from the CPU oracle.

Only the oracle (oracle/) and the seeded input generators
(paper_0704_3573_amd/inputs.py, which hold no Monte Carlo arithmetic) are
used; nothing here touches the HIP library.  Each fixture records, for the
seeded instance it names, what the oracle reaches after the stated number of
sweeps: energies and overlaps as integers, and 64-bit BLAKE2b digests of the
canonical spin, wheel and energy arrays (little-endian bytes of the arrays
exactly as the oracle returns them).

    python tests/golden/make_golden.py [c2 c3 c3all c4 c5 ...] [--threads N]

Workloads (the benchmark's configurations; sizes are the paper-shaped ones):
  c2     EA +-J, L = 64, 2 replicas, Metropolis T = 1.1, seed 2, 10^4 sweeps,
         E and Q after every 100 sweeps;
  c3     batched parallel tempering (L = 16, 24, 32, 48, 64 samples each,
         2 replicas x 32 temperatures 0.7..1.6, PT every 10 sweeps, seed
         3000): samples 5 and 63 of every L (all 64 copies of each) for 10^4
         sweeps, E by temperature and Q after every 1000 sweeps;
  c3all  the same workload, every copy of every sample, 100 sweeps;
  c4     q = 4 +-J Potts, heat bath T = 0.9, 2 replicas, seed 4000, 10^4
         sweeps, E and Q after every 100 sweeps: all 128 samples at L = 16,
         samples 0, 8, ..., 120 of the 128 at L = 32;
  c5     50 jobs of the serving stream (2000 jobs, arrivals seed 5, job seed
         5000 + j; every 40th job), each run alone to its requested sweeps.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_0704_3573_amd import inputs  # noqa: E402


def digest(a) -> str:
    """64-bit BLAKE2b digest (hex) of the little-endian bytes of an array."""
    a = np.ascontiguousarray(a)
    if a.dtype.byteorder == ">":
        a = a.astype(a.dtype.newbyteorder("<"))
    return hashlib.blake2b(a.tobytes(), digest_size=8).hexdigest()


def write(name, doc):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    print(f"wrote {path}", flush=True)


def sub_instance(inst, s, copies_per_sample, chains_per_sample):
    """Inputs of sample s of a job (a slice: the same arrays a one-sample job
    numbered from that sample would get)."""
    c0, h0 = s * copies_per_sample, s * chains_per_sample
    return {"J": inst["J"][s:s + 1], "spins": inst["spins"][c0:c0 + copies_per_sample],
            "wheels": inst["wheels"][c0:c0 + copies_per_sample],
            "ptwheels": inst["ptwheels"][h0:h0 + chains_per_sample]}


# ------------------------------------------------------------------ C2 ----
def make_c2(threads):
    L, T, n, me = 64, 1.1, 10_000, 100
    inst = inputs.make_instance("ising", L, 1, 2, 1, seed=2)
    t = time.time()
    out = oracle.run(oracle.ISING, oracle.METROPOLIS, L, [1 / T], inst["J"], inst["spins"],
                     inst["wheels"], n_replicas=2, n_sweeps=n, measure_every=me,
                     n_threads=min(threads, 2))
    write("c2_full.json", {
        "workload": "EA +-J L=64, 1 sample x 2 replicas, Metropolis T=1.1, seed 2",
        "sweeps": n, "measure_every": me, "oracle_seconds": round(time.time() - t, 1),
        "E_log": out["E_log"].tolist(), "Q_log": out["Q_log"].reshape(-1).tolist(),
        "E": out["E"].tolist(),
        "spins": [digest(out["spins"][c]) for c in range(2)],
        "wheels": [digest(out["wheels"][c]) for c in range(2)]})


# ------------------------------------------------------------------ C3 ----
C3_L = (16, 24, 32, 48)
C3_S, C3_R, C3_K, C3_PE, C3_SEED = 64, 2, 32, 10, 3000


def c3_betas():
    return 1.0 / inputs.linear_temperatures(C3_K, 0.7, 1.6)


def make_c3(threads):
    n, me = 10_000, 1000
    recs = []
    for i, L in enumerate(C3_L):
        for s in (5, 63):
            inst = inputs.make_instance("ising", L, 1, C3_R, C3_K, seed=C3_SEED,
                                        sample0=C3_S * i + s)
            t = time.time()
            out = oracle.run(oracle.ISING, oracle.METROPOLIS, L, c3_betas(), inst["J"],
                             inst["spins"], inst["wheels"], inst["ptwheels"], n_replicas=C3_R,
                             n_sweeps=n, pt_every=C3_PE, measure_every=me, n_threads=threads)
            recs.append({
                "L": L, "job_sample": s, "oracle_seconds": round(time.time() - t, 1),
                "E_log": out["E_log"].tolist(), "Q_log": out["Q_log"].reshape(n // me, -1).tolist(),
                "E": out["E"].tolist(), "slot_of_temp": out["slot_of_temp"].tolist(),
                "pt_accepts": out["pt_accepts"].tolist(),
                "spins": [digest(out["spins"][c]) for c in range(C3_R * C3_K)],
                "wheels": [digest(out["wheels"][c]) for c in range(C3_R * C3_K)],
                "ptwheels": [digest(out["ptwheels"][h]) for h in range(C3_R)]})
            print(f"c3 L={L} sample {s}: {recs[-1]['oracle_seconds']} s", flush=True)
    write("c3_chains.json", {
        "workload": "batched PT: 64 samples per L in (16, 24, 32, 48), 2 replicas x 32 "
                    "temperatures 0.7..1.6, Metropolis, PT every 10 sweeps, seed 3000 "
                    "(sample index 64 * job + s)",
        "sweeps": n, "measure_every": me, "records": recs})


def make_c3all(threads):
    n = 100
    jobs = []
    for i, L in enumerate(C3_L):
        inst = inputs.make_instance("ising", L, C3_S, C3_R, C3_K, seed=C3_SEED, sample0=C3_S * i)
        t = time.time()
        out = oracle.run(oracle.ISING, oracle.METROPOLIS, L, c3_betas(), inst["J"], inst["spins"],
                         inst["wheels"], inst["ptwheels"], n_samples=C3_S, n_replicas=C3_R,
                         n_sweeps=n, pt_every=C3_PE, n_threads=threads)
        cps, hps = C3_R * C3_K, C3_R
        per = []
        for s in range(C3_S):
            c = slice(s * cps, (s + 1) * cps)
            h = slice(s * hps, (s + 1) * hps)
            per.append({"spins": digest(out["spins"][c]), "wheels": digest(out["wheels"][c]),
                        "E": digest(out["E"][c]), "slot_of_temp": digest(out["slot_of_temp"][h]),
                        "ptwheels": digest(out["ptwheels"][h])})
        jobs.append({"L": L, "oracle_seconds": round(time.time() - t, 1), "samples": per,
                     "E_sum": int(out["E"].sum())})
        print(f"c3all L={L}: {jobs[-1]['oracle_seconds']} s", flush=True)
        del inst, out
    write("c3_all_copies.json", {
        "workload": "batched PT as in c3_chains.json, every copy of all 256 samples",
        "sweeps": n, "jobs": jobs})


# ------------------------------------------------------------------ C4 ----
def make_c4(threads):
    n, me, T, S, R = 10_000, 100, 0.9, 128, 2
    out_jobs = []
    for L, samples in ((16, list(range(S))), (32, list(range(0, S, 8)))):
        inst = inputs.make_instance("potts", L, S, R, 1, seed=4000)

        def one(s):
            sub = sub_instance(inst, s, R, R)
            out = oracle.run(oracle.POTTS, oracle.HEATBATH, L, [1 / T], sub["J"], sub["spins"],
                             sub["wheels"], n_replicas=R, n_sweeps=n, measure_every=me,
                             n_threads=2)
            return {"sample": s, "E": out["E"].tolist(), "Q": int(out["Q_log"][-1, 0, 0]),
                    "E_log": digest(out["E_log"]), "Q_log": digest(out["Q_log"].reshape(-1)),
                    "spins": digest(out["spins"]), "wheels": digest(out["wheels"])}

        t = time.time()
        with cf.ThreadPoolExecutor(max(1, threads // 2)) as ex:
            recs = list(ex.map(one, samples))
        out_jobs.append({"L": L, "oracle_seconds": round(time.time() - t, 1), "records": recs})
        print(f"c4 L={L}: {out_jobs[-1]['oracle_seconds']} s", flush=True)
    write("c4_potts.json", {
        "workload": "q=4 +-J Potts, 128 samples x 2 replicas, heat bath T=0.9, seed 4000; "
                    "E_log [n/100][2] and Q_log [n/100] digests",
        "sweeps": n, "measure_every": me, "jobs": out_jobs})


# ------------------------------------------------------------------ C5 ----
C5_JOBS, C5_EVERY = 2000, 40


def c5_sampled():
    """Every 40th job of the 2000-job serving stream (parameters do not depend
    on the arrival rate)."""
    return inputs.job_stream(C5_JOBS, 1.0, seed=5)[::C5_EVERY]


def make_c5(threads):
    jobs = c5_sampled()

    def one(p):
        model = oracle.ISING if p["model"] == "ising" else oracle.POTTS
        algo = oracle.METROPOLIS if p["model"] == "ising" else oracle.HEATBATH
        inst = inputs.make_instance(p["model"], p["L"], 1, 2, 1, p["seed"])
        out = oracle.run(model, algo, p["L"], [1.0 / p["T"]], inst["J"], inst["spins"],
                         inst["wheels"], n_replicas=2, n_sweeps=p["sweeps"],
                         measure_every=p["sweeps"], n_threads=2)
        r = {k: p[k] for k in ("rid", "model", "L", "T", "sweeps", "seed")}
        r.update({"E": out["E_log"][0].reshape(-1).tolist(), "Q": int(out["Q_log"][0, 0, 0]),
                  "spins": digest(out["spins"]), "wheels": digest(out["wheels"])})
        return r

    t = time.time()
    # longest jobs first so that the pool drains evenly
    order = sorted(range(len(jobs)), key=lambda j: -jobs[j]["L"] ** 3 * jobs[j]["sweeps"])
    with cf.ThreadPoolExecutor(max(1, threads // 2)) as ex:
        res = dict(zip(order, ex.map(one, [jobs[j] for j in order])))
    write("c5_sampled_jobs.json", {
        "workload": "serving stream: 2000 jobs (arrivals seed 5, job seed 5000 + j), every "
                    "40th job run alone; Ising -> Metropolis, Potts -> heat bath, 2 replicas",
        "oracle_seconds": round(time.time() - t, 1),
        "jobs": [res[j] for j in range(len(jobs))]})


MAKERS = {"c2": make_c2, "c3": make_c3, "c3all": make_c3all, "c4": make_c4, "c5": make_c5}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("which", nargs="*", default=list(MAKERS))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    oracle.lib()
    for w in a.which:
        MAKERS[w](a.threads)


if __name__ == "__main__":
    main()
