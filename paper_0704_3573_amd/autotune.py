"""Autotuner for the fused batched launch.

Both knobs are result-invariant: they fix the launch shape, never which
random number a site receives, so every candidate gives bit-identical
trajectories.

- Lanes per Parisi-Rapuano wheel of the 3D Potts jobs at L = 16 (eight or
  four, sec. 3.3's several numbers per wheel and step): eight fill more SIMDs
  when the batch is small, four spend fewer instructions per update when the
  device is full.  Tried first, at the automatic block size.
- Threads per workgroup of the fused sweep launch (a multiple of 64 between
  the largest per-copy wheel count of the batch and 1024): how many complete
  copies share one workgroup and its LDS, hence occupancy and idle lanes.

Each candidate is timed over a few periods of the batch itself (timing mode:
HIP events around the fused sweep launch); those periods advance the jobs
like any other sweeps.  The choice per batch signature (the multiset of
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


def lane_choices(jobs):
    """The jobs whose lanes per wheel may change, and the values to try."""
    js = [j for j in jobs if j.model in (B.POTTS, B.GPOTTS) and j.L == 16]
    return js, ([8, 4] if js else [])


def _set_lanes(jobs, lanes, stream):
    for j in jobs:
        j.set_wheel_lanes(lanes, stream)


def _time(batch, sweeps_per_period, periods, stream):
    batch.run(sweeps_per_period, stream)  # builds the plan, warms up
    ms = []
    for _ in range(periods):
        batch.run(sweeps_per_period, stream)
        ms.append(batch.sweep_ms())
    return min(ms)


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
    """Choose and set the lanes per wheel and the block size of `batch`;
    returns (block, {block: ms})."""
    sig = signature(batch.jobs)
    cache = _load(cache_path) if use_cache else {}
    ljobs, choices = lane_choices(batch.jobs)
    if sig in cache:
        if cache[sig].get("lanes") and ljobs:
            _set_lanes(ljobs, int(cache[sig]["lanes"]), stream)
        batch.set_block(int(cache[sig]["block"]))
        return int(cache[sig]["block"]), cache[sig].get("times", {})
    times, lanes = {}, None
    batch.set_timing(True)
    try:
        if len(choices) > 1:
            batch.set_block(0)
            lane_ms = {}
            for S in choices:
                _set_lanes(ljobs, S, stream)
                lane_ms[S] = _time(batch, sweeps_per_period, periods, stream)
            lanes = min(lane_ms, key=lane_ms.get)
            _set_lanes(ljobs, lanes, stream)
        for tpb in candidates(batch.jobs):
            try:
                batch.set_block(tpb)
                times[tpb] = _time(batch, sweeps_per_period, periods, stream)
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
        cache[sig] = {"block": best, "times": {str(k): v for k, v in times.items()}, "lanes": lanes}
        _save(cache_path, cache)
    return best, times
