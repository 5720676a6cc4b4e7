"""Equilibration analysis of measured overlaps (host side, numpy).

The library returns integer overlaps per (sample, temperature) at every
measurement (`Job.measure`); sec. 4.1 of the paper judges thermalisation from
them in three ways, built here on arrays of measurements:

* the Monte Carlo history of the squared overlap q^2 (sample average per
  measurement and temperature);
* log2 data binning: the measurements are cut into the last half, the
  quarter before it, the eighth before that and the sixteenth before that;
  q^2 is averaged over each group and all samples (with the standard error
  over samples) -- from the smallest group to the largest the averages
  should approach the equilibrium value;
* the overlap distribution P(q) on the overlap's integer support, and its
  asymmetry (half the L1 distance between P(q) and P(-q)), which vanishes at
  equilibrium for the Ising glass without a field.

Normalised overlaps: Ising glass q = Q / N; Ising-like models of Eq. 2
q = Q / N_occ over the sample's occupied sites; q = 4 Potts models
q = (4 C / N - 1) / 3 with C the number of equal sites.
"""
from __future__ import annotations

import numpy as np

ISING, POTTS, GPOTTS, ISING_GEN = 0, 1, 2, 3


def stack_measurements(Q_list, n_samples: int, n_temps: int) -> np.ndarray:
    """Measurements as returned by `Job.measure` (each [S*K]) -> int64
    [n_meas][S][K]."""
    return np.asarray(Q_list, dtype=np.int64).reshape(len(Q_list), n_samples, n_temps)


def sites_per_sample(model: int, L: int, J=None) -> np.ndarray:
    """Sites the overlap runs over, per sample: L^3, or the occupied sites of
    each sample of an Ising-like job (canonical couplings [S][5][N])."""
    if model == ISING_GEN:
        J = np.asarray(J)
        return (J[:, 3] == 1).sum(axis=1).astype(np.int64)
    S = 1 if J is None else np.asarray(J).shape[0]
    return np.full(S, L ** 3, dtype=np.int64)


def normalised_overlap(model: int, Q: np.ndarray, N: np.ndarray) -> np.ndarray:
    """q of every measurement; Q [n][S][K], N [S]."""
    Nf = np.asarray(N, dtype=np.float64)[None, :, None]
    if model in (POTTS, GPOTTS):
        return (4.0 * Q / Nf - 1.0) / 3.0
    return Q / Nf


def q2_history(model: int, Q: np.ndarray, N: np.ndarray) -> np.ndarray:
    """[n][K]: sample average of q^2 at every measurement."""
    q = normalised_overlap(model, Q, N)
    return (q * q).mean(axis=1)


def log2_groups(n: int):
    """(start, end) of the last half, previous quarter, previous eighth and
    previous sixteenth of n measurements, largest group first."""
    return [(n >> (j + 1), n >> j) for j in range(4)]


def log2_binning(model: int, Q: np.ndarray, N: np.ndarray):
    """Means [4][K] of q^2 per group (largest first) over the group's
    measurements and all samples, and their standard errors [4][K] over
    samples."""
    q = normalised_overlap(model, Q, N)
    q2 = q * q
    S = q2.shape[1]
    means, errs = [], []
    for lo, hi in log2_groups(q2.shape[0]):
        if hi <= lo:
            means.append(np.full(q2.shape[2], np.nan))
            errs.append(np.full(q2.shape[2], np.nan))
            continue
        per_sample = q2[lo:hi].mean(axis=0)  # [S][K]
        means.append(per_sample.mean(axis=0))
        errs.append(per_sample.std(axis=0, ddof=1) / np.sqrt(S) if S > 1
                    else np.full(q2.shape[2], np.nan))
    return np.array(means), np.array(errs)


def pq_counts(model: int, Q: np.ndarray, N: np.ndarray, start: int = 0) -> np.ndarray:
    """int64 [K][bins]: histogram of the overlap on its integer support over
    measurements start..end and all samples.  Ising models: bin Q + Nmax in
    0..2 Nmax (bins v and 2 Nmax - v hold Q and -Q); Potts: bin C in 0..N."""
    Nmax = int(np.max(N))
    potts = model in (POTTS, GPOTTS)
    nb = Nmax + 1 if potts else 2 * Nmax + 1
    vals = Q[start:] if potts else Q[start:] + Nmax  # [n'][S][K]
    K = Q.shape[2]
    out = np.zeros((K, nb), dtype=np.int64)
    for k in range(K):
        out[k] = np.bincount(vals[:, :, k].ravel(), minlength=nb)
    return out


def pq_asymmetry(counts: np.ndarray, bands: int | None = None) -> np.ndarray:
    """Per temperature: half the L1 distance between P(q) and P(-q) (Ising
    models).  With `bands`, both sides are first summed over `bands` equal
    bands of |Q| (band floor(|Q| bands / (N + 1)); Q = 0 on neither side), so
    that sparse histograms compare meaningfully."""
    tot = counts.sum(axis=1)
    if bands is None:
        diff = np.abs(counts - counts[:, ::-1]).sum(axis=1) / 2.0
    else:
        N = (counts.shape[1] - 1) // 2
        band = np.arange(1, N + 1) * bands // (N + 1)
        plus = np.zeros((counts.shape[0], bands), dtype=np.int64)
        minus = np.zeros_like(plus)
        for k in range(counts.shape[0]):
            plus[k] = np.bincount(band, weights=counts[k, N + 1:], minlength=bands)
            minus[k] = np.bincount(band, weights=counts[k, N - 1::-1], minlength=bands)
        diff = np.abs(plus - minus).sum(axis=1)  # each mirror pair of bands once
    return np.where(tot > 0, diff / np.maximum(tot, 1), 0.0)
