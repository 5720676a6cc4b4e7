"""Pins of the oracle's sweep: closed forms, invariants, exact enumeration.

* beta = 0: Metropolis flips every site every half-sweep (threshold 2^32);
  heat bath sets s = +1 exactly when r < 2^31; Potts picks r >> 30.  The
  last two tie each site to its documented random number (wheel (z, row
  group), colour-major, row, increasing x), so they pin the visit order.
* beta -> infinity: the energy never increases; a ferromagnetic ground state
  is a fixed point.
* Gauge covariance of Metropolis: acceptance depends only on the number of
  unsatisfied bonds, which a gauge transformation leaves unchanged.
* Energy bookkeeping: the energy tracked through the updates equals the
  energy recomputed from scratch after every sweep.
* L = 2 exact enumeration: the one-sweep transition matrix, built from the
  oracle's own site update, leaves the Boltzmann distribution of Eq. (1)
  invariant; long runs reproduce its energy histogram (also with parallel
  tempering, whose joint law is a product of Boltzmann laws).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_0704_3573_amd import inputs

TWO32 = 1 << 32


def draw_index_map(L):
    """(wheel, draw number within one sweep) of every site, by the convention."""
    rho = min(8, L)
    wheel = np.zeros(L ** 3, np.int64)
    pos = np.zeros(L ** 3, np.int64)
    for g in range(L // rho):
        for z in range(L):
            w = g * L + z
            k = 0
            for p in (0, 1):
                for y in range(g * rho, g * rho + rho):
                    for x in range(L):
                        if (x + y + z) % 2 == p:
                            i = x + L * (y + L * z)
                            wheel[i], pos[i] = w, k
                            k += 1
    return wheel, pos


def site_numbers(wheels, L, sweeps):
    """Random number used by every site in each of `sweeps` sweeps."""
    rho = min(8, L)
    per = rho * L
    wmap, pmap = draw_index_map(L)
    streams = np.stack([oracle.pr_stream(wheels[w], per * sweeps) for w in range(wheels.shape[0])])
    return np.stack([streams[wmap, t * per + pmap] for t in range(sweeps)])


@pytest.mark.parametrize("L", [2, 4, 8, 16])
def test_metropolis_beta_zero_flips_everything(L):
    inst = inputs.make_instance("ising", L, 1, 1, 1, seed=21)
    assert int(oracle.tables_metropolis(0.0)[0]) == TWO32
    s0 = inst["spins"][0]
    for t in (1, 2, 5):
        out = oracle.run(oracle.ISING, oracle.METROPOLIS, L, [0.0], inst["J"], inst["spins"],
                         inst["wheels"], n_sweeps=t)
        assert np.array_equal(out["spins"][0], s0 * (-1) ** t)


@pytest.mark.parametrize("L", [2, 4, 8, 24])
def test_heatbath_beta_zero_spins_are_msb_stream(L):
    inst = inputs.make_instance("ising", L, 1, 1, 1, seed=22)
    sweeps = 3
    r = site_numbers(inst["wheels"][0], L, sweeps)
    out = oracle.run(oracle.ISING, oracle.HEATBATH, L, [0.0], inst["J"], inst["spins"],
                     inst["wheels"], n_sweeps=sweeps)
    want = np.where(r[-1] < (1 << 31), 1, -1).astype(np.int8)
    assert np.array_equal(out["spins"][0], want)


@pytest.mark.parametrize("L", [2, 4, 8, 16])
def test_potts_beta_zero_states_are_top_bits(L):
    inst = inputs.make_instance("potts", L, 1, 1, 1, seed=23)
    sweeps = 2
    r = site_numbers(inst["wheels"][0], L, sweeps)
    out = oracle.run(oracle.POTTS, oracle.HEATBATH, L, [0.0], inst["J"], inst["spins"],
                     inst["wheels"], n_sweeps=sweeps)
    assert np.array_equal(out["spins"][0], (r[-1] >> 30).astype(np.uint8))


def test_wheels_advance_by_one_number_per_site():
    L = 8
    inst = inputs.make_instance("ising", L, 1, 1, 1, seed=24)
    out = oracle.run(oracle.ISING, oracle.METROPOLIS, L, [1.0], inst["J"], inst["spins"],
                     inst["wheels"], n_sweeps=3)
    per = min(8, L) * L
    for w in (0, 3, 7):
        seq = oracle.pr_stream(inst["wheels"][0, w], 3 * per + 100)
        nxt = oracle.pr_stream(out["wheels"][0, w], 100)
        assert np.array_equal(seq[3 * per:], nxt)


@pytest.mark.parametrize("algo", [oracle.METROPOLIS, oracle.HEATBATH])
def test_zero_temperature_energy_never_increases(algo):
    L = 8
    inst = inputs.make_instance("ising", L, 1, 1, 1, seed=25)
    beta = 60.0  # all thresholds are 0 or 2^32
    st, wh = inst["spins"], inst["wheels"]
    E = oracle.energy(oracle.ISING, L, st[0], inst["J"][0])
    for _ in range(30):
        out = oracle.run(oracle.ISING, algo, L, [beta], inst["J"], st, wh, n_sweeps=1)
        assert out["E"][0] <= E
        E, st, wh = out["E"][0], out["spins"], out["wheels"]


def test_ferromagnetic_ground_state_is_a_fixed_point():
    L = 8
    J = np.ones((1, 3, L ** 3), np.int8)
    for algo in (oracle.METROPOLIS, oracle.HEATBATH):
        s = np.ones((1, L ** 3), np.int8)
        wh = inputs.wheel_seeds(26, [0], oracle.wheels_per_copy(L))
        out = oracle.run(oracle.ISING, algo, L, [40.0], J, s, wh, n_sweeps=20)
        assert np.all(out["spins"] == 1) and out["E"][0] == -3 * L ** 3
    p = np.full((1, L ** 3), 2, np.uint8)
    out = oracle.run(oracle.POTTS, oracle.HEATBATH, L, [40.0], J, p, wh, n_sweeps=20)
    assert np.all(out["spins"] == 2) and out["E"][0] == -3 * L ** 3


def test_mattis_model_reaches_ground_state_at_low_temperature():
    L = 4
    xi = inputs.ising_spins(27, [99], L)[0].astype(np.int8)
    s3 = xi.reshape(L, L, L)
    J = np.stack([(s3 * np.roll(s3, -1, axis=ax)).reshape(-1) for ax in (2, 1, 0)])[None]
    inst = inputs.make_instance("ising", L, 1, 1, 1, seed=27)
    out = oracle.run(oracle.ISING, oracle.METROPOLIS, L, [3.0], J.astype(np.int8),
                     inst["spins"], inst["wheels"], n_sweeps=3000)
    assert out["E"][0] == -3 * L ** 3
    assert abs(int(np.sum(out["spins"][0] * xi))) == L ** 3


@pytest.mark.parametrize("L", [2, 4, 8])
def test_metropolis_gauge_covariance(L):
    inst = inputs.make_instance("ising", L, 1, 1, 1, seed=28)
    g = inputs.ising_spins(28, [1234], L)[0].astype(np.int8)
    g3 = g.reshape(L, L, L)
    J = inst["J"][0]
    Jg = np.stack([(J[d].reshape(L, L, L) * g3 * np.roll(g3, -1, axis=ax)).reshape(-1)
                   for d, ax in ((0, 2), (1, 1), (2, 0))]).astype(np.int8)
    st, sg = inst["spins"], inst["spins"] * g
    wh_a = wh_b = inst["wheels"]
    for t in range(15):
        a = oracle.run(oracle.ISING, oracle.METROPOLIS, L, [0.9], J[None], st, wh_a, n_sweeps=1)
        b = oracle.run(oracle.ISING, oracle.METROPOLIS, L, [0.9], Jg[None], sg, wh_b, n_sweeps=1)
        assert np.array_equal(b["spins"][0], a["spins"][0] * g)
        assert a["E"][0] == b["E"][0]
        st, sg, wh_a, wh_b = a["spins"], b["spins"], a["wheels"], b["wheels"]


@pytest.mark.parametrize("model,algo", [(oracle.ISING, oracle.METROPOLIS),
                                        (oracle.ISING, oracle.HEATBATH),
                                        (oracle.POTTS, oracle.HEATBATH)])
@pytest.mark.parametrize("L", [2, 4, 8, 16])
def test_tracked_energy_equals_recomputed_every_sweep(model, algo, L):
    name = "ising" if model == oracle.ISING else "potts"
    inst = inputs.make_instance(name, L, 2, 1, 1, seed=29)
    oracle.run(model, algo, L, [1.0 / 1.1], inst["J"], inst["spins"], inst["wheels"],
               n_samples=2, n_sweeps=40, check_energy=True)


# ------------------------------------------------------ exact enumeration --

def l2_states():
    return np.array([[1 - 2 * ((m >> i) & 1) for i in range(8)] for m in range(256)], np.int8)


def l2_order():
    wmap, pmap = draw_index_map(2)
    # colour 0 before colour 1; sites of one colour do not interact
    return sorted(range(8), key=lambda i: ((sum(divmod(i, 2)) + i // 4) % 2, wmap[i], pmap[i]))


def site_kernel(L, algo, J, tab, i, states):
    n = states.shape[0]
    P = np.zeros((n, n))
    index = {bytes(s.tobytes()): k for k, s in enumerate(states)}
    for a, s in enumerate(states):
        # number of r values that end with s_i = -s_i (Metropolis) or +1 (heat bath)
        lo, hi = 0, TWO32
        while lo < hi:
            mid = (lo + hi) // 2
            u = s.copy()
            oracle.ising_update_site(L, algo, u, J, i, mid, tab)
            hit = (u[i] != s[i]) if algo == oracle.METROPOLIS else (u[i] == 1)
            if hit:
                lo = mid + 1
            else:
                hi = mid
        p = lo / TWO32
        t1 = s.copy()
        if algo == oracle.METROPOLIS:
            t1[i] = -s[i]
            P[a, index[t1.tobytes()]] += p
            P[a, a] += 1 - p
        else:
            t0 = s.copy()
            t1[i], t0[i] = 1, -1
            P[a, index[t1.tobytes()]] += p
            P[a, index[t0.tobytes()]] += 1 - p
    return P


@pytest.mark.parametrize("algo", [oracle.METROPOLIS, oracle.HEATBATH])
@pytest.mark.parametrize("T", [0.8, 1.5])
def test_l2_sweep_leaves_boltzmann_invariant(algo, T):
    L, beta = 2, 1.0 / T
    J = inputs.couplings(30, 0, L)
    states = l2_states()
    E = np.array([oracle.energy(oracle.ISING, L, s, J) for s in states], float)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    tab = oracle.tables_metropolis(beta) if algo == oracle.METROPOLIS else oracle.tables_heatbath(beta)
    P = np.eye(256)
    for i in l2_order():
        P = P @ site_kernel(L, algo, J, tab, i, states)
    assert np.allclose(P.sum(1), 1.0)
    assert np.max(np.abs(pi @ P - pi)) < 1e-8
    # and it is not trivially the identity
    assert np.max(np.abs(P - np.eye(256))) > 0.1


def exact_energy_law(J, beta, model=oracle.ISING):
    L = 2
    if model == oracle.ISING:
        states = l2_states()
    else:
        states = np.array(list(itertools.product(range(4), repeat=8)), np.uint8)
    E = np.array([oracle.energy(model, L, s, J) for s in states])
    w = np.exp(-beta * (E - E.min()))
    levels = np.unique(E)
    return levels, np.array([w[E == e].sum() for e in levels]) / w.sum()


def chi2_ok(samples, levels, probs, n_eff):
    counts = np.array([(samples == e).sum() for e in levels], float)
    assert counts.sum() == len(samples)
    expect = probs * len(samples)
    keep = expect > 20
    chi2 = ((counts[keep] - expect[keep]) ** 2 / expect[keep]).sum() * n_eff / len(samples)
    dof = keep.sum() - 1
    # normal approximation of the chi-square tail; 6 sigma is a fixed-seed guard
    return chi2 < dof + 6 * math.sqrt(2 * dof), chi2, dof


@pytest.mark.parametrize("model,algo", [(oracle.ISING, oracle.METROPOLIS),
                                        (oracle.ISING, oracle.HEATBATH),
                                        (oracle.POTTS, oracle.HEATBATH)])
def test_l2_long_run_energy_histogram(model, algo):
    L, beta = 2, 0.7
    name = "ising" if model == oracle.ISING else "potts"
    inst = inputs.make_instance(name, L, 1, 1, 1, seed=31)
    n = 200_000
    out = oracle.run(model, algo, L, [beta], inst["J"], inst["spins"], inst["wheels"],
                     n_sweeps=n, measure_every=2)
    levels, probs = exact_energy_law(inst["J"][0], beta, model)
    ok, chi2, dof = chi2_ok(out["E_log"][:, 0], levels, probs, n_eff=n // 2)
    assert ok, (chi2, dof)


def test_l2_parallel_tempering_marginals_are_boltzmann():
    L = 2
    betas = np.array([1.2, 0.8, 0.4])
    inst = inputs.make_instance("ising", L, 1, 1, 3, seed=32)
    n = 150_000
    out = oracle.run(oracle.ISING, oracle.METROPOLIS, L, betas, inst["J"], inst["spins"],
                     inst["wheels"], inst["ptwheels"], n_sweeps=n, pt_every=1, measure_every=3)
    assert out["pt_accepts"].min() > 0.05 * n
    for k, b in enumerate(betas):
        levels, probs = exact_energy_law(inst["J"][0], b)
        ok, chi2, dof = chi2_ok(out["E_log"][:, k], levels, probs, n_eff=n // 3)
        assert ok, (k, chi2, dof)


@pytest.mark.parametrize("model", ["ising_met", "ising_hb", "potts", "gpotts"])
@pytest.mark.parametrize("L", [4, 8])
def test_same_colour_updates_commute(model, L):
    """The checkerboard's race freedom (sec. 3.1), on the oracle's own site
    update: with every site of one colour given its own number, updating
    them in any order gives the same configuration, because no two sites
    of one colour are neighbours.  Updating sites of both colours in a
    different order does change the result (the test can see an order
    dependence when there is one)."""
    rng = np.random.default_rng(100 + L)
    N = L ** 3
    beta = 0.9
    J = rng.choice(np.array([-1, 1], np.int8), size=(3, N)).astype(np.int8)
    if model.startswith("ising"):
        s0 = rng.choice(np.array([-1, 1], np.int8), size=N).astype(np.int8)
        algo = oracle.METROPOLIS if model == "ising_met" else oracle.HEATBATH
        T = oracle.tables_metropolis(beta) if algo == oracle.METROPOLIS else oracle.tables_heatbath(beta)
        upd = lambda s, i, r: oracle.ising_update_site(L, algo, s, J, i, r, T)
    elif model == "potts":
        s0 = rng.integers(0, 4, N).astype(np.uint8)
        W = oracle.tables_potts(beta)
        upd = lambda s, i, r: oracle.potts_update_site(L, s, J, i, r, W)
    else:
        s0 = rng.integers(0, 4, N).astype(np.uint8)
        P = rng.integers(0, 24, (3, N)).astype(np.uint8)
        W = oracle.tables_potts(beta)
        upd = lambda s, i, r: oracle.gpotts_update_site(L, s, P, i, r, W)
    r = rng.integers(0, TWO32, N, dtype=np.uint64)
    x, y, z = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    colour = ((x + y + z) % 2).transpose(2, 1, 0).reshape(-1)  # site i = x + L (y + L z)
    for p in (0, 1):
        sites = np.flatnonzero(colour == p)
        a, b = s0.copy(), s0.copy()
        for i in sites:
            upd(a, int(i), int(r[i]))
        for i in rng.permutation(sites):
            upd(b, int(i), int(r[i]))
        assert np.array_equal(a, b), (model, L, p)
    # both colours: the order matters
    a, b = s0.copy(), s0.copy()
    for i in range(N):
        upd(a, i, int(r[i]))
    for i in rng.permutation(N):
        upd(b, int(i), int(r[i]))
    assert not np.array_equal(a, b)
