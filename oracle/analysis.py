"""Oracle of the equilibration analysis (test infrastructure only: imported by
tests/ and nothing else).

Sec. 4.1 of the paper checks thermalisation with three views of the replica
overlap: the Monte Carlo history of the squared overlap q^2, the log2 data
binning of the measurements (the last half, the quarter before it, the eighth
before that and the sixteenth before that, each averaged over all samples;
from the smallest group to the largest the averages should drift toward
equilibrium), and the overlap distribution P(q), symmetric at equilibrium
without a field.

Written as plain loops over the integer measurements in the order the paper
describes them.  Normalisations (the paper uses q^2 and P(q) without
defining them): Ising glass q = Q / N with Q = sum_i s^a_i s^b_i; Ising-like
models of Eq. 2 q = Q / N_occ over the occupied sites; q = 4 Potts models
the scalar overlap q = (4 C / N - 1) / 3 with C = sum_i delta(s^a_i, s^b_i).

Input layout: Q_log[t][s][k] = overlap of replicas 0 and 1 of sample s at
temperature index k in measurement t.
"""
import math

ISING, POTTS, GPOTTS, ISING_GEN = 0, 1, 2, 3


def overlap_q(model, Q, N):
    """Normalised overlap of one measurement (N: sites, or occupied sites for
    the Ising-like models)."""
    if model in (POTTS, GPOTTS):
        return (4.0 * Q / N - 1.0) / 3.0
    return Q / N


def q2_history(model, Q_log, N_of_sample):
    """[t][k]: the sample average of q^2 at every measurement."""
    out = []
    for row in Q_log:
        S, K = len(row), len(row[0])
        line = []
        for k in range(K):
            acc = 0.0
            for s in range(S):
                q = overlap_q(model, int(row[s][k]), N_of_sample[s])
                acc += q * q
            line.append(acc / S)
        out.append(line)
    return out


def log2_groups(n):
    """Measurement index ranges of the four groups, largest first: the last
    half, the previous quarter, the previous eighth, the previous sixteenth."""
    return [(n >> (j + 1), n >> j) for j in range(4)]


def log2_bins(model, Q_log, N_of_sample):
    """For each group (largest first) and temperature: (mean of q^2 over the
    group's measurements and all samples, standard error over samples of the
    per-sample group means)."""
    n = len(Q_log)
    S, K = len(Q_log[0]), len(Q_log[0][0])
    result = []
    for lo, hi in log2_groups(n):
        per_k = []
        for k in range(K):
            means = []
            for s in range(S):
                acc = 0.0
                for t in range(lo, hi):
                    q = overlap_q(model, int(Q_log[t][s][k]), N_of_sample[s])
                    acc += q * q
                means.append(acc / (hi - lo) if hi > lo else float("nan"))
            m = sum(means) / S
            var = sum((x - m) ** 2 for x in means) / (S - 1) if S > 1 else float("nan")
            per_k.append((m, math.sqrt(var / S) if S > 1 else float("nan")))
        result.append(per_k)
    return result


def pq_counts(model, Q_log, N_of_sample, start=0):
    """Histogram of the overlap on its integer support, per temperature, over
    measurements start..end and all samples.  Ising and Ising-like models:
    bin v = Q + N in 0..2N (N: the largest N over samples, so that bins v and
    2N - v hold Q and -Q); Potts: bin v = C in 0..N."""
    K = len(Q_log[0][0])
    Nmax = max(N_of_sample)
    potts = model in (POTTS, GPOTTS)
    counts = [[0] * (Nmax + 1 if potts else 2 * Nmax + 1) for _ in range(K)]
    for t in range(start, len(Q_log)):
        for row in Q_log[t]:
            for k in range(K):
                Q = int(row[k])
                counts[k][Q if potts else Q + Nmax] += 1
    return counts


def pq_asymmetry(counts, bands=None):
    """Half the L1 distance between P(q) and P(-q) for the Ising models (0:
    symmetric, 1: disjoint), per temperature.  With `bands`, the overlaps are
    first grouped by |Q| into that many equal bands on each side (band
    j = floor(|Q| bands / (N + 1))), so that a sparse histogram is compared
    band by band; Q = 0 belongs to neither side."""
    out = []
    for c in counts:
        tot = sum(c)
        n = len(c) - 1
        if not tot:
            out.append(0.0)
        elif bands is None:
            out.append(sum(abs(c[v] - c[n - v]) for v in range(n + 1)) / (2.0 * tot))
        else:
            N = n // 2
            plus, minus = [0] * bands, [0] * bands
            for v in range(n + 1):
                Q = v - N
                if Q > 0:
                    plus[Q * bands // (N + 1)] += c[v]
                elif Q < 0:
                    minus[-Q * bands // (N + 1)] += c[v]
            # each band of one side is compared once with its mirror band
            out.append(sum(abs(a - b) for a, b in zip(plus, minus)) / float(tot))
    return out
