"""Autotuner for the fused batched launch.

The only knob is result-invariant: the number of threads per workgroup of
the fused sweep launch (a multiple of 64 between the largest per-copy wheel
count of the batch and 1024).  It fixes how many complete copies share one
workgroup and its LDS, hence occupancy and idle lanes, but never which random
number a site receives, so every candidate gives bit-identical trajectories.

Each candidate is timed over a few periods of the batch itself (timing mode:
HIP events around the fused sweep launch); those periods advance the jobs
like any other sweeps.  The best block per batch signature (the multiset of
(model, algorithm, L, copies) of its jobs) is cached in a JSON file.
"""
from __future__ import annotations

import json
import os

from . import binding as B

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_0704_3573_amd",
                             "autotune.json")


def signature(jobs) -> str:
    parts = sorted(f"{j.model}:{j.algo}:{j.L}:{j.C}" for j in jobs)
    return ";".join(parts)


def candidates(jobs):
    lo = max(j.NW for j in jobs)
    lo = (lo + 63) // 64 * 64
    return list(range(lo, 1025, 64))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune(batch: B.Batch, sweeps_per_period: int, periods: int = 2, stream=None,
         cache_path: str = DEFAULT_CACHE, use_cache: bool = True):
    """Choose and set the block size of `batch`; returns (block, {block: ms})."""
    sig = signature(batch.jobs)
    cache = _load(cache_path) if use_cache else {}
    if sig in cache:
        batch.set_block(int(cache[sig]["block"]))
        return int(cache[sig]["block"]), cache[sig].get("times", {})
    times = {}
    batch.set_timing(True)
    try:
        for tpb in candidates(batch.jobs):
            try:
                batch.set_block(tpb)
                batch.run(sweeps_per_period, stream)  # builds the plan, warms up
                ms = []
                for _ in range(periods):
                    batch.run(sweeps_per_period, stream)
                    ms.append(batch.sweep_ms())
                times[tpb] = min(ms)
            except B.SgError:
                continue
    finally:
        batch.set_timing(False)
    if not times:
        batch.set_block(0)
        return batch.block(), times
    best = min(times, key=times.get)
    batch.set_block(best)
    if use_cache:
        cache[sig] = {"block": best, "times": {str(k): v for k, v in times.items()}}
        _save(cache_path, cache)
    return best, times
