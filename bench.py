#!/usr/bin/env python3
"""Benchmark: spin updates per nanosecond on one MI355X, batched and plain.

Headline (value): the batched parallel-tempering workload -- 256 disorder
samples of the 3D Edwards-Anderson +-J glass (64 each at L = 16, 24, 32, 48)
x 2 replicas x 32 temperatures (T = 0.7 .. 1.6 linear), Metropolis
checkerboard sweeps with a parallel-tempering step every 10 sweeps, all of
them advanced by one fused sweep launch per period replayed from a captured
hipGraph.  One step = one period: 10 sweeps of all 16384 copies (6.6e9
site updates) + the swap step.  Beside it, the plain single-lattice form
(L = 64, two replicas, T = 1.1, 100 sweeps + energy/overlap measurement per
step) and the CPU oracle timed on the host cores on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# int32 vector lanes: 256 CUs x 4 SIMD x 16 lanes per clock at 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# algorithmic integer operations per Metropolis site update: Eq. (5) draw
# (one add, one xor), one compare with the site's threshold, one operation
# recording the decision in the site's word, and the bit-sliced six-bond
# count with the flip amortised over the 32 sites of a word (about half an
# operation per site); the lower end of the 4.5 .. 8.5 operations the
# method needs per update
ALG_OPS_PER_UPDATE = 4.5
# Ising-like models (Eq. 2): the same plus one operation forming the site's
# threshold-table index (the paper's update cell reads a LUT in the same way)
GEN_ALG_OPS_PER_UPDATE = 5
C3_LS = (16, 24, 32, 48)
C3_SAMPLES_PER_L, C3_R, C3_K, C3_PT = 64, 2, 32, 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def c3_alg_bytes_per_update():
    # spins read + written once per launch of 10 sweeps is far below this;
    # per update the method touches its own bit and the six couplings, which
    # 64 copies of a sample share: 2 bits / 8 + 3 bits / (8 * 64)
    return 0.25 + 0.375 / (C3_R * C3_K)


# threads per workgroup of the rocprofv3 runs behind profiles/ising_sweep_c3_*
PROFILED_BLOCK = 512


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_0704_3573_amd", "csrc", "sg_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def committed_counters():
    """Values of the committed rocprofv3 counter summary of the batched sweep
    launch, if it was taken on the current kernel source (else {})."""
    p = os.path.join(ROOT, "profiles", "ising_sweep_c3_counters.txt")
    if not os.path.exists(p):
        return {}
    vals = {}
    for line in open(p):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return {}
    out = {}
    for k in ("hbm_bytes_per_launch", "valu_lane_ops_per_update", "valu_busy_fraction",
              "lds_bank_conflict_fraction"):
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return out


def build_c3(ctx, B, inputs, algo=None):
    algo = B.METROPOLIS if algo is None else algo
    jobs = []
    sample0 = 0
    betas = 1.0 / inputs.linear_temperatures(C3_K, 0.7, 1.6)
    for L in C3_LS:
        t = time.perf_counter()
        inst = inputs.make_instance("ising", L, C3_SAMPLES_PER_L, C3_R, C3_K, seed=3000,
                                    sample0=sample0)
        jobs.append(B.Job(ctx, B.ISING, algo, L, betas, inst["J"], inst["spins"],
                          inst["wheels"], inst["ptwheels"], n_samples=C3_SAMPLES_PER_L,
                          n_replicas=C3_R, pt_every=C3_PT))
        del inst
        sample0 += C3_SAMPLES_PER_L
        log(f"[bench] job L={L}: {C3_SAMPLES_PER_L * C3_R * C3_K} copies ready in "
            f"{time.perf_counter() - t:.1f}s")
    return jobs


def c5_mean_updates_per_job():
    """Mean site updates of a job of the serving workload: 2 replicas x L^3
    (L uniform in {8,16,24,32,48}) x 10^U sweeps (U uniform in [3, 5])."""
    import math
    e_sites = 2 * sum(L ** 3 for L in (8, 16, 24, 32, 48)) / 5
    e_sweeps = (10 ** 5 - 10 ** 3) / (2 * math.log(10))
    return e_sites * e_sweeps


def serving_bench(ctx, n_jobs=2000, cap_s=60.0, calib_s=3.0, seed=5):
    """Continuous-batching request loop on the serving workload: Poisson jobs,
    EA Ising (Metropolis) or q=4 Potts (heat bath) with probability 1/2, L
    uniform in {8,16,24,32,48}, T uniform in [0.7, 1.6], 2 replicas, sweeps
    floor(10^U[3,5]), job seed 5000 + j, arrivals seed 5, admitted by HBM
    budget and slots.  The saturated capacity is measured first: 2 n_jobs
    jobs of the same distribution arrive at once, so that every slot stays
    taken; the updates performed between 1.5 s (the slots are filled by then)
    and 1.5 + calib_s seconds of wall clock give the capacity, and the stream then
    arrives at 1.2x that capacity (jobs/s = updates/ns / mean updates per
    job).  The stream (n_jobs jobs, about 1.4e9 updates each) runs until it
    is served or for cap_s seconds of wall clock: jobs arrived, started and
    completed, latency percentiles of the completed ones, all updates
    performed per ns, and the share of the wall clock with a period on the
    device."""
    from paper_0704_3573_amd import serving
    mean_upd = c5_mean_updates_per_job()
    be = serving.DeviceBackend(ctx)
    burst = serving.poisson_stream(2 * n_jobs, rate=0.0, seed=seed + 1, seed0=9000)
    srv = serving.Server(be, hbm_budget=64 << 30, max_slots=512)
    srv.serve(burst, cap_s=1.5)
    u0, t = srv.updates_done(), time.perf_counter()
    srv.serve([], cap_s=calib_s)
    wall = time.perf_counter() - t
    cap_ups = (srv.updates_done() - u0) / (wall * 1e9)
    cap_jobs = cap_ups * 1e9 / mean_upd
    rate = 1.2 * cap_jobs
    host = {k: round(v, 3) for k, v in srv.host_s.items()}
    log(f"[bench] serving capacity: {cap_ups:.1f} updates/ns over {wall:.1f}s with "
        f"{len(srv.active)} of 512 slots taken at the end ({srv.periods} periods, "
        f"{srv.changes} membership changes, host seconds {host}) -> {cap_jobs:.3f} jobs/s")
    srv.release()
    reqs = serving.poisson_stream(n_jobs, rate=rate, seed=seed)
    srv = serving.Server(be, hbm_budget=64 << 30, max_slots=512)
    be.busy = []
    t = time.perf_counter()
    done = srv.serve(reqs, cap_s=cap_s)
    wall = time.perf_counter() - t
    busy_s = be.busy_seconds()
    be.close()
    arrived = sum(1 for r in reqs if r.arrival <= wall)
    out = serving.summary(done, wall, updates=srv.updates_done())
    out.update({"capacity_updates_per_ns": round(cap_ups, 3),
                "capacity_jobs_per_s": round(cap_jobs, 4), "arrival_rate_per_s": round(rate, 4),
                "cap_s": cap_s, "jobs_in_stream": n_jobs, "jobs_arrived": arrived,
                "jobs_started": arrived - len(srv.pending) - len(srv.creating),
                "jobs_completed": len(done), "peak_resident_jobs": srv.peak_slots,
                "membership_changes": srv.changes,
                "periods": srv.periods, "device_busy_share": round(busy_s / wall, 4),
                "mean_updates_per_job": round(mean_upd, -6),
                "latency_note": "percentiles over the jobs completed within the cap",
                "workload": f"{n_jobs} Poisson jobs, Ising-Metropolis/Potts-heat-bath 1:1, "
                            "L in {8,16,24,32,48}, T~U[0.7,1.6], sweeps 10^U[3,5], 2 replicas, "
                            "HBM budget 64 GiB, 512 slots, rate 1.2x the measured capacity, "
                            f"{cap_s:.0f} s wall-clock cap"})
    srv.release()
    return out


def cpu_baseline(budget_s=15.0):
    """The oracle on a bounded sample of the batched workload: one sample of
    each L with its 64 copies, whole parallel-tempering periods."""
    import numpy as np

    import oracle
    from paper_0704_3573_amd import inputs
    threads = max(1, min(16, os.cpu_count() or 1))
    betas = 1.0 / inputs.linear_temperatures(C3_K, 0.7, 1.6)
    insts = [inputs.make_instance("ising", L, 1, C3_R, C3_K, seed=3000, sample0=i * 64)
             for i, L in enumerate(C3_LS)]
    updates, elapsed, periods = 0, 0.0, 0
    while elapsed < budget_s and periods < 50:
        for L, inst in zip(C3_LS, insts):
            t = time.perf_counter()
            out = oracle.run(oracle.ISING, oracle.METROPOLIS, L, betas, inst["J"], inst["spins"],
                             inst["wheels"], inst["ptwheels"], n_samples=1, n_replicas=C3_R,
                             n_sweeps=C3_PT, pt_every=C3_PT, n_threads=threads)
            elapsed += time.perf_counter() - t
            updates += C3_PT * C3_R * C3_K * L ** 3
            inst["spins"], inst["wheels"], inst["ptwheels"] = (out["spins"], out["wheels"],
                                                               out["ptwheels"])
        periods += 1
    # single thread, the plain workloads: EA L = 8 (1 replica, 1000 sweeps,
    # whole run) and EA L = 64 with two replicas (a 50-sweep sample of the
    # 10^4-sweep run), Metropolis at T = 1.1
    single = {}
    for name, L, R, n in (("L8_1000_sweeps", 8, 1, 1000), ("L64_2_replicas_50_sweeps", 64, 2, 50)):
        inst = inputs.make_instance("ising", L, 1, R, 1, seed=1 if L == 8 else 2)
        t = time.perf_counter()
        oracle.run(oracle.ISING, oracle.METROPOLIS, L, [1 / 1.1], inst["J"], inst["spins"],
                   inst["wheels"], n_replicas=R, n_sweeps=n, n_threads=1)
        dt = time.perf_counter() - t
        ups = R * L ** 3 * n
        single[name] = {"ns_per_update": round(dt * 1e9 / ups, 3),
                        "updates_per_ns": round(ups / (dt * 1e9), 5)}
    del np
    return {"value": updates / (elapsed * 1e9), "unit": "spin updates/ns", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"one sample per L in {list(C3_LS)} with its {C3_R * C3_K} copies "
                      f"(2 replicas x 32 temperatures), {periods} parallel-tempering period(s) "
                      f"of {C3_PT} sweeps each, {updates:.3g} updates in {elapsed:.1f}s",
            "single_thread": single}


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def heat_bath_c3(ctx, B, inputs, np, torch, stream, steps, block):
    """The batched parallel-tempering workload with heat-bath dynamics (Eq. 4)
    instead of Metropolis: same samples, temperatures and PT period, the
    fused launch at the Metropolis run's block size; wall clock per step and
    HIP-event time of the sweep launch."""
    jobs = build_c3(ctx, B, inputs, B.HEATBATH)
    batch = B.Batch(ctx, jobs, block=block)
    for _ in range(3):
        batch.run(C3_PT, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run(C3_PT, stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    batch.set_timing(True)
    batch.run(C3_PT, stream)
    batch.sweep_ms()
    kms = []
    for _ in range(10):
        batch.run(C3_PT, stream)
        kms.append(batch.sweep_ms())
    sites = sum(j.C * j.N for j in jobs)
    out = {"value": round(C3_PT * sites / (ms * 1e6), 3), "unit": "spin updates/ns",
           "ms_per_step": round(ms, 4), "kernel_ms_per_launch": round(float(np.mean(kms)), 4),
           "block_threads": block,
           "workload": "the batched workload (256 EA samples at L=16,24,32,48 x 2 replicas x 32 "
                       "temperatures, PT every 10 sweeps) with heat-bath dynamics"}
    log(f"[bench] heat bath: {out}")
    return out


def potts_c4(ctx, B, inputs, np, torch, stream, sweeps, model="potts"):
    """q = 4 Potts heat bath, 128 samples x 2 replicas: updates/ns over
    periods of `sweeps` sweeps (one launch each), wall clock and HIP-event
    kernel time.  model "potts": the +-J glass at T = 0.9, L = 16 and 32;
    "gpotts": the glassy (permutation) model of Eq. 3 at beta = 2.4, the
    paper's 3D Potts temperature, L = 16 and 32; "gpotts4": the glassy model
    in 4D at beta = 1.405, the paper's 4D temperature, L = 16."""
    out = {}
    mid, beta, seed, Ls = {"potts": (B.POTTS, 1 / 0.9, 4000, (16, 32)),
                           "gpotts": (B.GPOTTS, 2.4, 4100, (16, 32)),
                           "gpotts4": (B.GPOTTS4, 1.405, 4600, (16,))}[model]
    for L in Ls:
        inst = inputs.make_instance(model, L, 128, 2, 1, seed=seed)
        job = B.Job(ctx, mid, B.HEATBATH, L, [beta], inst["J"], inst["spins"],
                    inst["wheels"], n_samples=128, n_replicas=2)
        del inst
        pb = B.Batch(ctx, [job])
        pb.run(sweeps, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            pb.run(sweeps, stream)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3 / 3
        pb.set_timing(True)
        pk = []
        for _ in range(3):
            pb.run(sweeps, stream)
            pk.append(pb.sweep_ms())
        ups = job.C * job.N * sweeps
        out[f"L{L}"] = {"value": round(ups / (wall_ms * 1e6), 3), "unit": "spin updates/ns",
                        "ms_per_period": round(wall_ms, 3),
                        "kernel_ms_per_period": round(float(np.mean(pk)), 3),
                        "block_threads": pb.block()}
        log(f"[bench] {model} L={L}: {wall_ms:.2f} ms per {sweeps} sweeps, "
            f"{out[f'L{L}']['value']:.1f} updates/ns")
        del pb, job
    if model == "potts":
        out["workload"] = (f"q=4 +-J Potts glass, 128 samples x 2 replicas, heat bath T=0.9, "
                           f"period = {sweeps} sweeps (one launch)")
    elif model == "gpotts4":
        out["workload"] = (f"q=4 glassy Potts model (Eq. 3) on the 4D hypercubic lattice, L=16, "
                           f"128 samples x 2 replicas, heat bath beta=1.405, period = {sweeps} "
                           f"sweeps (one launch)")
        # the paper's 4D glassy Potts rates (L = 16): 64 ps/spin (LX200),
        # 125 ps/spin (LX160), 150 ns/spin (PC)
        out["paper_updates_per_ns"] = {"Virtex4-LX200": 15.625, "Virtex4-LX160": 8.0,
                                       "PC": round(1 / 150, 5)}
    else:
        out["workload"] = (f"q=4 glassy Potts model (random permutation couplings, Eq. 3), "
                           f"128 samples x 2 replicas, heat bath beta=2.4, period = {sweeps} "
                           f"sweeps (one launch)")
        # the paper's 3D glassy Potts rates (L = 16): 64 ps/spin (LX200),
        # 125 ps/spin (LX160), 117 ns/spin (PC)
        out["paper_updates_per_ns"] = {"Virtex4-LX200": 15.625, "Virtex4-LX160": 8.0,
                                       "PC": round(1 / 117, 5)}
    return out


def ising_like(ctx, B, inputs, np, torch, stream, sweeps):
    """Ising-like models of Eq. 2, Metropolis, no parallel tempering: the
    random-field Ising model (J = +1, h_i = +-1.5) and the diluted
    antiferromagnet in a field (J = -1, h = 1.0, each site occupied with
    probability 1/2), at L = 32 (64 samples x 2 replicas x 16 temperatures)
    and L = 64 (16 samples x 2 replicas x 8 temperatures), T = 1.0 .. 4.0.
    Updates/ns over periods of `sweeps` sweeps (one launch each), wall clock
    and HIP-event kernel time; empty sites count as visited sites."""
    out = {}
    for kind, h, seed in (("rfim", 1.5, 4300), ("daff", 1.0, 4400)):
        for L, S, K in ((32, 64, 16), (64, 16, 8)):
            betas = [1.0 / (1.0 + 3.0 * k / (K - 1)) for k in range(K)]
            inst = inputs.make_instance(kind, L, S, 2, K, seed=seed)
            job = B.Job(ctx, B.ISING_GEN, B.METROPOLIS, L, betas, inst["J"], inst["spins"],
                        inst["wheels"], n_samples=S, n_replicas=2, field=h)
            del inst
            pb = B.Batch(ctx, [job])
            pb.run(sweeps, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                pb.run(sweeps, stream)
            torch.cuda.synchronize()
            wall_ms = (time.perf_counter() - t0) * 1e3 / 3
            pb.set_timing(True)
            pk = []
            for _ in range(3):
                pb.run(sweeps, stream)
                pk.append(pb.sweep_ms())
            kms = float(np.mean(pk))
            ups = job.C * job.N * sweeps
            key = f"{kind}_L{L}"
            out[key] = {"value": round(ups / (wall_ms * 1e6), 3), "unit": "spin updates/ns",
                        "copies": job.C, "ms_per_period": round(wall_ms, 3),
                        "kernel_ms_per_period": round(kms, 3),
                        "kernel_updates_per_ns": round(ups / (kms * 1e6), 3),
                        "alu_frac": round(ups * GEN_ALG_OPS_PER_UPDATE / (kms * 1e-3) / 1e12
                                          / VALU_PEAK_TOPS, 4),
                        "block_threads": pb.block()}
            log(f"[bench] {kind} L={L}: {wall_ms:.2f} ms per {sweeps} sweeps, "
                f"{out[key]['value']:.1f} updates/ns")
            del pb, job
    out["workload"] = (f"Ising-like models of Eq. 2, Metropolis: RFIM |h|=1.5 and DAFF h=1.0 "
                       f"(occupation 1/2); L=32: 64 samples x 2 replicas x 16 temperatures, "
                       f"L=64: 16 x 2 x 8, T=1.0..4.0; period = {sweeps} sweeps (one launch)")
    out["alg_ops_per_update"] = GEN_ALG_OPS_PER_UPDATE
    return out


def equilibration(ctx, B, inputs, np, torch, stream, n_meas):
    """Equilibration analysis of sec. 4.1 on a measured run: EA glass L = 16,
    16 samples x 2 replicas x 8 temperatures T = 0.7 .. 1.6, Metropolis, PT
    every 10 sweeps, overlaps measured after every PT period (n_meas
    measurements); q^2 log2 bins and P(q) asymmetry from the library's
    analysis module, and the cost of measuring (run time with the
    measurements vs the same sweeps without)."""
    from paper_0704_3573_amd import analysis as A
    L, S, K, every = 16, 16, 8, 10
    temps = np.linspace(0.7, 1.6, K)
    inst = inputs.make_instance("ising", L, S, 2, K, seed=4500)
    mk = lambda: B.Job(ctx, B.ISING, B.METROPOLIS, L, 1.0 / temps, inst["J"], inst["spins"],
                       inst["wheels"], inst["ptwheels"], n_samples=S, n_replicas=2,
                       pt_every=every)
    job = mk()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_meas):
        job.sweep(every, stream)
    torch.cuda.synchronize()
    bare_s = time.perf_counter() - t0
    del job
    job = mk()
    Qs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_meas):
        job.sweep(every, stream)
        Qs.append(job.measure(stream)[1])
    meas_s = time.perf_counter() - t0
    t1 = time.perf_counter()
    Q = A.stack_measurements(Qs, S, K)
    N = A.sites_per_sample(A.ISING, L, inst["J"])
    means, errs = A.log2_binning(A.ISING, Q, N)
    asym = A.pq_asymmetry(A.pq_counts(A.ISING, Q, N, start=n_meas // 2), bands=16)
    analysis_ms = (time.perf_counter() - t1) * 1e3
    ups = n_meas * every * job.C * job.N
    out = {"workload": f"EA +-J L={L}, {S} samples x 2 replicas x {K} temperatures "
                       f"T=0.7..1.6, Metropolis, PT every {every} sweeps, overlaps after every "
                       f"period, {n_meas} measurements ({n_meas * every} sweeps)",
           "updates_per_ns_with_measurements": round(ups / (meas_s * 1e9), 3),
           "updates_per_ns_without": round(ups / (bare_s * 1e9), 3),
           "measurement_overhead": round(meas_s / bare_s - 1.0, 4),
           "analysis_ms": round(analysis_ms, 3),
           "q2_log2_bins_T0.7": [round(float(x), 5) for x in means[::-1, 0]],
           "q2_log2_bins_T1.6": [round(float(x), 5) for x in means[::-1, -1]],
           "q2_log2_bins_order": "sixteenth, eighth, quarter, last half",
           "pq_asymmetry_last_half_16_bands": [round(float(x), 4) for x in asym]}
    log(f"[bench] equilibration: {out}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed batched steps (10 sweeps each)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=5,
                    help="timed plain steps (100 sweeps + measurement each)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--serving-jobs", type=int, default=2000,
                    help="jobs in the serving stream (0 = skip the serving measurement)")
    ap.add_argument("--serving-cap", type=float, default=60.0,
                    help="wall-clock seconds the serving stream runs for")
    ap.add_argument("--serving-only", action="store_true",
                    help="time only the serving workload (profiling runs)")
    ap.add_argument("--potts-sweeps", type=int, default=200,
                    help="sweeps per timed Potts period (0 = skip the Potts measurement)")
    ap.add_argument("--gen-sweeps", type=int, default=50,
                    help="sweeps per timed Ising-like (RFIM, DAFF) period (0 = skip)")
    ap.add_argument("--gen-only", action="store_true",
                    help="time only the Ising-like workload (profiling runs)")
    ap.add_argument("--eq-meas", type=int, default=256,
                    help="measurements of the equilibration-analysis run (0 = skip)")
    ap.add_argument("--no-heat-bath", dest="heat_bath", action="store_false",
                    help="skip the heat-bath run of the batched workload")
    ap.add_argument("--no-tune", action="store_true", help="skip the block-size autotuner")
    ap.add_argument("--block", type=int, default=0,
                    help="force the fused launch's threads per workgroup (skips the tuner)")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched form (profiling runs)")
    ap.add_argument("--potts-only", action="store_true",
                    help="time only the Potts heat-bath workload (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): this build has no "
              "multi-GPU path; independent samples would be sharded one job set per GPU.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0704_3573_amd import binding as B
    from paper_0704_3573_amd import inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calibration} MiB x 5")
        return
    ctx = B.Context(0)
    stream = torch.cuda.current_stream()

    if args.serving_only:
        log(f"[bench] serving only: {serving_bench(ctx, args.serving_jobs, args.serving_cap)}")
        return

    if args.gen_only:
        log(f"[bench] Ising-like only: {ising_like(ctx, B, inputs, np, torch, stream, args.gen_sweeps)}")
        return

    if args.potts_only:
        log(f"[bench] Potts only: {potts_c4(ctx, B, inputs, np, torch, stream, args.potts_sweeps)}")
        log("[bench] glassy Potts only: "
            f"{potts_c4(ctx, B, inputs, np, torch, stream, args.potts_sweeps, 'gpotts')}")
        log("[bench] 4D glassy Potts only: "
            f"{potts_c4(ctx, B, inputs, np, torch, stream, args.potts_sweeps, 'gpotts4')}")
        return

    # ------------------------------------------------ batched (headline) --
    jobs = build_c3(ctx, B, inputs)
    batch = B.Batch(ctx, jobs)
    tune_times = {}
    if args.block:
        batch.set_block(args.block)
    elif not args.no_tune:
        from paper_0704_3573_amd import autotune
        tpb, tune_times = autotune.tune(batch, C3_PT, periods=5, stream=stream, use_cache=False)
        # keep the block the committed counter summary was taken on unless
        # another one is clearly faster (within 3 % they tie: 512 and 1024
        # differ by about 1 %, and run-to-run noise reaches 1.5 %)
        if tpb != PROFILED_BLOCK and tune_times.get(PROFILED_BLOCK, float("inf")) <= 1.03 * tune_times[tpb]:
            tpb = PROFILED_BLOCK
            batch.set_block(tpb)
        log(f"[bench] autotuned block: {tpb} threads "
            f"({', '.join(f'{k}:{v:.3f}ms' for k, v in sorted(tune_times.items()))})")
    tpb = batch.block()
    sites = sum(j.C * j.N for j in jobs)
    log(f"[bench] batched: {len(jobs)} jobs, {sum(j.C for j in jobs)} copies, {sites} sites, "
        f"block {tpb} threads")
    for _ in range(args.warmup):
        batch.run(C3_PT, stream)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run(C3_PT, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    updates_per_step = C3_PT * sites
    value = updates_per_step / (ms_per_step * 1e6)
    log(f"[bench] batched: {ms_per_step:.3f} ms/step, {value:.1f} updates/ns")

    # live kernel timing: HIP events recorded inside the replayed graph around
    # the fused sweep launch (same stream, same graph)
    batch.set_timing(True)
    batch.run(C3_PT, stream)
    batch.sweep_ms()
    kms = []
    for _ in range(max(5, min(args.steps, 50))):
        batch.run(C3_PT, stream)
        kms.append(batch.sweep_ms())
    batch.set_timing(False)
    kernel_ms = float(np.mean(kms))
    achieved = updates_per_step * ALG_OPS_PER_UPDATE / (kernel_ms * 1e-3) / 1e12
    counters = committed_counters()
    traffic = counters.get("hbm_bytes_per_launch")
    log(f"[bench] sweep kernel: {kernel_ms:.3f} ms per launch ({C3_PT} sweeps), "
        f"{achieved:.2f} TOP/s algorithmic")
    E = [j.energies() for j in jobs]
    e_per_site = float(np.mean(np.concatenate([e / j.N for e, j in zip(E, jobs)])))
    del batch, jobs
    if args.batched_only:
        log(f"[bench] batched only: {value:.1f} updates/ns")
        return

    hb = heat_bath_c3(ctx, B, inputs, np, torch, stream, args.steps, tpb) \
        if args.heat_bath else None

    # --------------------------------------------------------- plain form --
    L2 = 64
    inst = inputs.make_instance("ising", L2, 1, 2, 1, seed=2)
    job = B.Job(ctx, B.ISING, B.METROPOLIS, L2, [1 / 1.1], inst["J"], inst["spins"],
                inst["wheels"], n_samples=1, n_replicas=2)
    job.sweep(100, stream)
    job.measure(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.plain_steps):
        job.sweep(100, stream)
        job.measure(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain_ms = (t1 - t0) * 1e3 / args.plain_steps
    plain_value = 100 * 2 * L2 ** 3 / (plain_ms * 1e6)
    log(f"[bench] plain: {plain_ms:.1f} ms per 100 sweeps + measurement, "
        f"{plain_value:.2f} updates/ns")
    del job

    # ------------------------------------------- q = 4 Potts, heat bath --
    potts = potts_c4(ctx, B, inputs, np, torch, stream, args.potts_sweeps) \
        if args.potts_sweeps > 0 else None
    glassy = potts_c4(ctx, B, inputs, np, torch, stream, args.potts_sweeps, "gpotts") \
        if args.potts_sweeps > 0 else None
    glassy4d = potts_c4(ctx, B, inputs, np, torch, stream, args.potts_sweeps, "gpotts4") \
        if args.potts_sweeps > 0 else None

    isinglike = ising_like(ctx, B, inputs, np, torch, stream, args.gen_sweeps) \
        if args.gen_sweeps > 0 else None

    eq = equilibration(ctx, B, inputs, np, torch, stream, args.eq_meas) \
        if args.eq_meas > 0 else None

    serving_stats = None
    if args.serving_jobs > 0:
        serving_stats = serving_bench(ctx, args.serving_jobs, args.serving_cap)
        log(f"[bench] serving: {serving_stats}")

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(args.cpu_budget)
        log(f"[bench] CPU oracle: {cpu['value']:.4f} updates/ns on {cpu['cores']} threads")

    line = {
        "metric": "spin updates/ns on 1 MI355X (plain vs batched), bit-exact; % HBM roofline",
        "value": round(value, 3),
        "unit": "spin updates/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded +-J couplings, spins and wheel seeds)",
        "config": {
            "workload": "batched parallel tempering: 256 EA +-J samples (64 each at L=16,24,32,48)"
                        " x 2 replicas x 32 temperatures T=0.7..1.6, Metropolis, PT every 10 "
                        "sweeps; step = 10 sweeps + PT step",
            "copies": 16384, "sites": sites, "updates_per_step": updates_per_step,
            "block_threads": tpb, "parallelism": "single GPU",
            "autotune_ms_per_launch": {str(k): round(v, 4) for k, v in sorted(tune_times.items())},
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "TOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": traffic,
            "kernel": "ising_sweep_kernel<Metropolis>",
            "kernel_ms_per_launch": round(kernel_ms, 4),
            "alg_ops_per_update": ALG_OPS_PER_UPDATE,
            "hbm_alg_bytes_per_update": round(c3_alg_bytes_per_update(), 4),
            "hbm_frac_alg": round(value * c3_alg_bytes_per_update() / HBM_PEAK_GBS, 5),
            # measured (committed rocprofv3 counters of this kernel source):
            # HBM bytes per launch over the live launch time, and the VALU
            # lane-operations issued per update and the VALU issue fraction
            "hbm_gbs_measured": None if traffic is None else round(traffic / (kernel_ms * 1e-3) / 1e9, 1),
            "hbm_frac_measured": None if traffic is None else
            round(traffic / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "valu_lane_ops_per_update_measured": counters.get("valu_lane_ops_per_update"),
            "valu_issue_frac_measured": counters.get("valu_busy_fraction"),
            "lds_bank_conflict_frac_measured": counters.get("lds_bank_conflict_fraction"),
        },
        "plain": {
            "value": round(plain_value, 3),
            "unit": "spin updates/ns",
            "workload": "EA +-J L=64, 2 replicas, T=1.1, Metropolis; step = 100 sweeps + E,Q",
            "ms_per_step": round(plain_ms, 3),
        },
        "speedup_batched_over_plain": round(value / plain_value, 2),
        "heat_bath": hb,
        "potts_c4": potts,
        "glassy_potts": glassy,
        "glassy_potts_4d": glassy4d,
        "ising_like": isinglike,
        "equilibration": eq,
        "serving": serving_stats,
        "cpu_baseline": cpu,
        "context": {"paper_fpga_ea_updates_per_ns": {"Virtex4-LX160": 31.25,
                                                     "Virtex4-LX200": 62.5},
                    "mean_energy_per_site": round(e_per_site, 4)},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
