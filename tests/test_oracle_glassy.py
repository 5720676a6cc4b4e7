"""Pins of the oracle's glassy (permutation) Potts model, Eq. (3):
H = -sum_<ij> delta(s_i, pi_ij(s_j)), q = 4, heat bath.

* Gauge invariance of the energy: relabelling the states of every site by a
  permutation tau_i and the couplings by pi_ij -> tau_i pi_ij tau_j^-1 maps
  every term delta(s_i, pi_ij(s_j)) to itself, so the energy is unchanged.
  Reading the term the other way round (delta(s_j, pi(s_i))) breaks it.
* Local fields are energy differences: h_a - h_b = E(s_i = b) - E(s_i = a),
  for the bonds stored at i and at its three lower neighbours alike.
* Identity couplings give the ferromagnetic q = 4 Potts model: a run with
  every pi = identity equals the +-J Potts run with every J = +1 (a separate
  code path, pinned on its own), state by state and number by number.
* beta = 0: every weight is 2^28, so the new state is the top two bits of the
  site's number (ties the visits to the documented draw order).
* L = 2 exact enumeration (4^8 states): long heat-bath runs reproduce the
  Boltzmann energy law of Eq. (1).
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_0704_3573_amd import inputs
from tests.test_oracle_dynamics import chi2_ok, exact_energy_law, site_numbers

PERMS = [tuple(p) for p in itertools.permutations(range(4))]


def images(byte):
    return tuple((int(byte) >> (2 * v)) & 3 for v in range(4))


def to_byte(p):
    return sum(p[v] << (2 * v) for v in range(4))


def compose(f, g):
    """(f o g)(v) = f(g(v))."""
    return tuple(f[g[v]] for v in range(4))


def inverse(p):
    out = [0] * 4
    for v in range(4):
        out[p[v]] = v
    return tuple(out)


def site(L, x, y, z):
    return (x % L) + L * ((y % L) + L * (z % L))


def gauge(L, s, P, tau):
    """Relabel states by tau_i and couplings by tau_i pi tau_j^-1 (bond i -> i + e_d)."""
    N = L ** 3
    s2 = np.array([tau[i][s[i]] for i in range(N)], np.uint8)
    P2 = np.zeros_like(P)
    for z in range(L):
        for y in range(L):
            for x in range(L):
                i = site(L, x, y, z)
                for d, j in enumerate((site(L, x + 1, y, z), site(L, x, y + 1, z),
                                       site(L, x, y, z + 1))):
                    pi = images(P[d, i])
                    P2[d, i] = to_byte(compose(tau[i], compose(pi, inverse(tau[j]))))
    return s2, P2


def test_permutation_bytes_are_the_24_permutations():
    pb = inputs.permutation_bytes()
    assert sorted(images(b) for b in pb) == sorted(PERMS)
    assert images(pb[0]) == (0, 1, 2, 3)
    J = inputs.glassy_couplings(5, 0, 8)
    assert J.shape == (3, 512) and J.dtype == np.uint8
    assert set(np.unique(J)) <= set(pb.tolist())
    # all 24 occur, roughly uniformly (1536 bonds, 64 expected each)
    counts = np.array([(J == b).sum() for b in pb])
    assert counts.min() > 30 and counts.max() < 110


@pytest.mark.parametrize("L", [2, 4])
def test_energy_is_gauge_invariant(L):
    rng = np.random.default_rng(L)
    inst = inputs.make_instance("gpotts", L, 1, 1, 1, seed=40 + L)
    P, s = inst["J"][0], inst["spins"][0]
    E = oracle.energy(oracle.GPOTTS, L, s, P)
    for trial in range(3):
        tau = [PERMS[k] for k in rng.integers(0, 24, L ** 3)]
        s2, P2 = gauge(L, s, P, tau)
        assert oracle.energy(oracle.GPOTTS, L, s2, P2) == E
    # a reading with the roles of i and j exchanged is not invariant
    def swapped_energy(s, P):
        e = 0
        for z in range(L):
            for y in range(L):
                for x in range(L):
                    i = site(L, x, y, z)
                    for d, j in enumerate((site(L, x + 1, y, z), site(L, x, y + 1, z),
                                           site(L, x, y, z + 1))):
                        e -= int(s[j] == images(P[d, i])[s[i]])
        return e
    assert any(swapped_energy(*gauge(L, s, P, [PERMS[k] for k in rng.integers(0, 24, L ** 3)]))
               != swapped_energy(s, P) for _ in range(5))


@pytest.mark.parametrize("L", [2, 4])
def test_fields_are_energy_differences(L):
    inst = inputs.make_instance("gpotts", L, 1, 1, 1, seed=50 + L)
    P, s = inst["J"][0], inst["spins"][0].copy()
    for i in range(L ** 3):
        h = oracle.gpotts_fields(L, s, P, i)
        assert h.min() >= 0 and h.sum() <= 6
        E = []
        for a in range(4):
            t = s.copy()
            t[i] = a
            E.append(oracle.energy(oracle.GPOTTS, L, t, P))
        for a in range(4):
            for b in range(4):
                assert h[a] - h[b] == E[b] - E[a], (i, a, b)


def test_identity_couplings_equal_the_ferromagnetic_potts_model():
    L, n = 4, 6
    inst = inputs.make_instance("gpotts", L, 2, 2, 1, seed=60)
    ident = np.full_like(inst["J"], inputs.permutation_bytes()[0])
    ferro = np.ones(inst["J"].shape, np.int8)
    for T in (0.6, 1.3):
        a = oracle.run(oracle.GPOTTS, oracle.HEATBATH, L, [1 / T], ident, inst["spins"],
                       inst["wheels"], n_samples=2, n_replicas=2, n_sweeps=n, check_energy=True)
        b = oracle.run(oracle.POTTS, oracle.HEATBATH, L, [1 / T], ferro, inst["spins"],
                       inst["wheels"], n_samples=2, n_replicas=2, n_sweeps=n)
        assert np.array_equal(a["spins"], b["spins"])
        assert np.array_equal(a["wheels"], b["wheels"])
        assert np.array_equal(a["E"], b["E"])
    # a generic instance differs from the ferromagnet
    g = oracle.run(oracle.GPOTTS, oracle.HEATBATH, L, [1 / 0.6], inst["J"], inst["spins"],
                   inst["wheels"], n_samples=2, n_replicas=2, n_sweeps=n)
    assert not np.array_equal(g["spins"], a["spins"])


@pytest.mark.parametrize("L", [2, 4, 8])
def test_beta_zero_states_are_top_bits(L):
    inst = inputs.make_instance("gpotts", L, 1, 1, 1, seed=70)
    out = oracle.run(oracle.GPOTTS, oracle.HEATBATH, L, [0.0], inst["J"], inst["spins"],
                     inst["wheels"], n_sweeps=1)
    r = site_numbers(inst["wheels"][0], L, 1)[0]
    assert np.array_equal(out["spins"][0], (r >> 30).astype(np.uint8))


@pytest.mark.parametrize("L", [2, 4, 8])
def test_tracked_energy_equals_recomputed_every_sweep(L):
    inst = inputs.make_instance("gpotts", L, 2, 1, 1, seed=80)
    oracle.run(oracle.GPOTTS, oracle.HEATBATH, L, [1 / 0.9], inst["J"], inst["spins"],
               inst["wheels"], n_samples=2, n_sweeps=30, check_energy=True)


@pytest.mark.parametrize("beta", [0.7, 1.4])
def test_l2_long_run_energy_histogram(beta):
    L = 2
    inst = inputs.make_instance("gpotts", L, 1, 1, 1, seed=90)
    n = 200_000
    out = oracle.run(oracle.GPOTTS, oracle.HEATBATH, L, [beta], inst["J"], inst["spins"],
                     inst["wheels"], n_sweeps=n, measure_every=2)
    levels, probs = exact_energy_law(inst["J"][0], beta, oracle.GPOTTS)
    assert len(levels) >= 5
    ok, chi2, dof = chi2_ok(out["E_log"][:, 0], levels, probs, n_eff=n // 2)
    assert ok, (chi2, dof)
