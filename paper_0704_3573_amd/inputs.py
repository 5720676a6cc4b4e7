"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module holds no Monte Carlo arithmetic.  It only turns a 64-bit seed
into the quenched disorder, the initial configurations and the external
random values that initialise every Parisi-Rapuano wheel (the paper's
section 3.3 says the wheels are loaded with externally generated random
values; section 2.1 defines +-1 couplings for the Edwards-Anderson glass).

Generator: SplitMix64 (Steele, Lea and Flood, 2014), used as a counter-based
stream.  Output u of a stream with key K is mix64(K + (u+1) * GOLDEN), where
mix64 is the SplitMix64 finaliser.  Stream keys are derived from
(seed, tag, a, b) by the same finaliser, so every array is a pure function of
its indices and can be regenerated piecewise.

Encodings (canonical, host side):
  * site index i = x + L*(y + L*z), periodic cubic lattice of side L;
  * couplings J: int8 array [3][N], J[d][i] joins i and i + e_d (d = x, y, z);
    bit b of stream output u gives element 64*u + b, bit 1 -> -1;
  * glassy-Potts couplings (permutations of 0..3, Eq. 3): uint8 [3][N], the
    bond joining i and i + e_d holds the permutation pi of its term
    delta(s_i, pi(s_{i+e_d})) as its images, pi(v) = (byte >> 2v) & 3; element
    n is permutation number (stream output n mod 24) in lexicographic order;
  * the 4D glassy Potts model ("gpotts4"): hypercubic lattice of side L,
    site i = x + L*(y + L*(z + L*u)), N = L^4, couplings uint8 [4][N] (d = x,
    y, z, u) on a stream of their own, spins as for Potts; one sweep wheel per
    (z, u, group of rho rows), L * L * L / rho per copy;
  * Ising-like models of Eq. 2 (dilution x_i, field h_i = |h| f_i): int8
    [5][N], rows J_x, J_y, J_z, x, f.  "rfim": J = +1, x = 1, f iid +-1;
    "daff": J = -1, x iid in {0, 1} (p = 1/2), f = +1; "isinggen": J, x and
    f all iid (+-1, {0, 1}, +-1).  x and f use the bit rule of the couplings
    (bit 1 -> x = 0, f = -1) on streams of their own;
  * Ising spins: int8 +-1, same bit rule;  Potts spins: uint8 0..3, two bits
    per site (bits 2k, 2k+1 of the stream word, little end first);
  * wheel seeds: 61 uint32 words per wheel, oldest first, I(-61) .. I(-1),
    each the high 32 bits of one stream output; bit 0 of I(-1) is forced to 1
    so the low-bit lagged-Fibonacci sequence is never all even.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

TAG_J = 0x4A  # 'J' couplings
TAG_S = 0x53  # 'S' initial spins
TAG_W = 0x57  # 'W' sweep wheels
TAG_P = 0x50  # 'P' parallel-tempering wheels
TAG_Q = 0x51  # 'Q' glassy-Potts permutation couplings
TAG_X = 0x58  # 'X' dilution
TAG_F = 0x46  # 'F' field signs


def mix64(z):
    """SplitMix64 finaliser on uint64 numpy values (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, tag: int, a=0, b=0):
    """Key of the stream (seed, tag, a, b); a and b may be numpy arrays."""
    with np.errstate(over="ignore"):
        k = mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + np.uint64(tag) * GOLDEN)
        k = mix64(k ^ (np.asarray(a, dtype=np.uint64) + np.uint64(1)) * _M1)
        k = mix64(k ^ (np.asarray(b, dtype=np.uint64) + np.uint64(1)) * _M2)
    return k


def stream(key, n: int):
    """n outputs of each stream in `key` (shape key.shape + (n,))."""
    key = np.asarray(key, dtype=np.uint64)
    u = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key[..., None] + u * GOLDEN)


def _bits(key, nbits: int):
    """Bits of the streams in `key`, bit b of output u at position 64 u + b."""
    words = stream(key, (nbits + 63) // 64).astype("<u8")
    bits = np.unpackbits(words.view(np.uint8), axis=-1, bitorder="little")
    return bits[..., :nbits]


def couplings(seed: int, sample: int, L: int) -> np.ndarray:
    """int8 [3][L^3] +-1 couplings of one disorder sample (iid, p = 1/2)."""
    n = L ** 3
    b = _bits(stream_key(seed, TAG_J, sample), 3 * n)
    return (1 - 2 * b.astype(np.int8)).reshape(3, n)


def permutation_bytes() -> np.ndarray:
    """uint8 [24]: the permutations of (0, 1, 2, 3) in lexicographic order,
    each as the byte pi(0) | pi(1) << 2 | pi(2) << 4 | pi(3) << 6."""
    import itertools
    return np.array([sum(p[v] << (2 * v) for v in range(4))
                     for p in itertools.permutations(range(4))], dtype=np.uint8)


def glassy_couplings(seed: int, sample: int, L: int, dim: int = 3) -> np.ndarray:
    """uint8 [dim][L^dim] iid uniform random permutations, one per bond
    (3D and 4D draw from different streams)."""
    n = L ** dim
    key = stream_key(seed, TAG_Q, sample) if dim == 3 else stream_key(seed, TAG_Q, sample, dim)
    u = stream(key, dim * n) % np.uint64(24)
    return permutation_bytes()[u.astype(np.int64)].reshape(dim, n)


def ising_like_couplings(kind: str, seed: int, sample: int, L: int) -> np.ndarray:
    """int8 [5][L^3]: J_x, J_y, J_z, x, f of one sample of an Ising-like
    model of Eq. 2 ("rfim", "daff" or "isinggen")."""
    n = L ** 3
    out = np.empty((5, n), np.int8)
    bx = _bits(stream_key(seed, TAG_X, sample), n).astype(np.int8)
    bf = _bits(stream_key(seed, TAG_F, sample), n).astype(np.int8)
    if kind == "rfim":
        out[:3], out[3], out[4] = 1, 1, 1 - 2 * bf
    elif kind == "daff":
        out[:3], out[3], out[4] = -1, 1 - bx, 1
    elif kind == "isinggen":
        out[:3], out[3], out[4] = couplings(seed, sample, L), 1 - bx, 1 - 2 * bf
    else:
        raise ValueError(kind)
    return out


def ising_spins(seed: int, copies, L: int) -> np.ndarray:
    """int8 [len(copies)][L^3] iid +-1 initial spins."""
    copies = np.atleast_1d(np.asarray(copies, dtype=np.uint64))
    b = _bits(stream_key(seed, TAG_S, copies), L ** 3)
    return (1 - 2 * b.astype(np.int8))


def potts_spins(seed: int, copies, L: int, q: int = 4, dim: int = 3) -> np.ndarray:
    """uint8 [len(copies)][L^dim] iid initial Potts states in 0..3 (q = 4)."""
    if q != 4:
        raise ValueError("only q = 4 has a two-bit encoding")
    copies = np.atleast_1d(np.asarray(copies, dtype=np.uint64))
    n = L ** dim
    b = _bits(stream_key(seed, TAG_S, copies), 2 * n)
    b = b.reshape(b.shape[:-1] + (n, 2))
    return (b[..., 0] | (b[..., 1] << 1)).astype(np.uint8)


def _wheel_words(seed: int, tag: int, a, b):
    w = (stream(stream_key(seed, tag, a, b), 61) >> np.uint64(32)).astype(np.uint32)
    w[..., 60] |= np.uint32(1)
    return w


def wheel_seeds(seed: int, copies, n_wheels: int) -> np.ndarray:
    """uint32 [len(copies)][n_wheels][61]: I(-61)..I(-1) of every sweep wheel."""
    copies = np.atleast_1d(np.asarray(copies, dtype=np.uint64))
    w = np.arange(n_wheels, dtype=np.uint64)
    return _wheel_words(seed, TAG_W, copies[:, None], w[None, :])


def pt_wheel_seeds(seed: int, chains) -> np.ndarray:
    """uint32 [len(chains)][61]: seed words of each parallel-tempering wheel."""
    chains = np.atleast_1d(np.asarray(chains, dtype=np.uint64))
    return _wheel_words(seed, TAG_P, chains, 0)


def rho(L: int) -> int:
    """Rows of one z-plane served by one wheel: min(8, L)."""
    return min(8, L)


def wheels_per_copy(L: int, dim: int = 3) -> int:
    """One wheel per (z, group of rho rows): L * L / rho; in 4D one per
    (z, u, group of rho rows): L^3 / rho."""
    return L ** (dim - 2) * (L // rho(L))


def make_instance(model: str, L: int, n_samples: int, n_replicas: int,
                  n_temps: int, seed: int, sample0: int = 0):
    """All inputs of one job: couplings, spins, sweep wheels, PT wheels.
    model: "ising", "potts" (+-J Potts glass), "gpotts" (glassy Potts),
    "gpotts4" (glassy Potts in 4D, J [S][4][L^4]), or an Ising-like model of
    Eq. 2: "rfim", "daff", "isinggen" (J is then [S][5][N]).

    Copy (slot) c = (s * R + r) * K + k for sample s, replica r, slot k.
    Samples are numbered from `sample0` so that one large campaign can be
    split into several jobs without changing any sample's inputs.
    """
    S, R, K = n_samples, n_replicas, n_temps
    C = S * R * K
    dim = 4 if model == "gpotts4" else 3
    if model == "gpotts":
        make_J = glassy_couplings
    elif model == "gpotts4":
        def make_J(seed, sample, L):
            return glassy_couplings(seed, sample, L, dim=4)
    elif model in ("rfim", "daff", "isinggen"):
        def make_J(seed, sample, L):
            return ising_like_couplings(model, seed, sample, L)
    else:
        make_J = couplings
    J = np.stack([make_J(seed, sample0 + s, L) for s in range(S)])
    glob = np.arange(C, dtype=np.uint64) + np.uint64(sample0 * R * K)
    if model in ("ising", "rfim", "daff", "isinggen"):
        sp = ising_spins(seed, glob, L)
    elif model in ("potts", "gpotts", "gpotts4"):
        sp = potts_spins(seed, glob, L, dim=dim)
    else:
        raise ValueError(model)
    wh = wheel_seeds(seed, glob, wheels_per_copy(L, dim))
    chains = np.arange(S * R, dtype=np.uint64) + np.uint64(sample0 * R)
    pw = pt_wheel_seeds(seed, chains)
    return {"J": np.ascontiguousarray(J), "spins": np.ascontiguousarray(sp),
            "wheels": np.ascontiguousarray(wh), "ptwheels": np.ascontiguousarray(pw)}


def linear_temperatures(K: int, t_min: float = 0.7, t_max: float = 1.6) -> np.ndarray:
    """Temperatures t_min + (t_max - t_min) * i / (K - 1), i = 0..K-1."""
    if K == 1:
        return np.array([t_min])
    i = np.arange(K, dtype=np.float64)
    return t_min + (t_max - t_min) * i / (K - 1)


def job_stream(n_jobs: int, rate: float, seed: int = 5, sweeps_lo: float = 3.0,
               sweeps_hi: float = 5.0, sizes=(8, 16, 24, 32, 48), t_range=(0.7, 1.6),
               seed0: int = 5000):
    """Parameters of a stream of simulation jobs: exponential inter-arrival
    times (rate per second), model "ising" (Metropolis) or "potts" (heat bath)
    with probability 1/2, L uniform in `sizes`, T uniform in t_range,
    sweeps = floor(10^U[sweeps_lo, sweeps_hi]), job seed seed0 + j.  Returns
    dicts with keys rid, model, L, T, sweeps, seed, arrival.  The job
    parameters do not depend on the rate."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0, size=n_jobs)
    t = np.cumsum(gaps / rate) if rate > 0 else np.zeros(n_jobs)
    out = []
    for j in range(n_jobs):
        out.append({"rid": j, "model": "ising" if rng.random() < 0.5 else "potts",
                    "L": int(rng.choice(sizes)), "T": float(rng.uniform(*t_range)),
                    "sweeps": int(np.floor(10 ** rng.uniform(sweeps_lo, sweeps_hi))),
                    "seed": seed0 + j, "arrival": float(t[j])})
    return out
