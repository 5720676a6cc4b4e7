"""CPU: the integer tables the library uploads equal the oracle's, bit for
bit (sec. 2.2 Metropolis rule, Eq. 4 heat bath, the Potts weights, the
parallel-tempering factors, and the 26 site classes of the Ising-like models
of Eq. 2).  Trajectory parity cannot see a threshold one unit off (a test
would have to draw exactly that number), so the tables are compared
directly, through the library's host-only export calls.
"""
import numpy as np
import pytest

import oracle
from paper_0704_3573_amd import binding as B
from paper_0704_3573_amd import inputs

TWO32 = 1 << 32
BETAS = [0.0, 1e-3, 0.05, 1 / 1.6, 1 / 1.1, 1 / 0.9, 1 / 0.7, 1.405, 2.4, 3.0, 20.0, 60.0]


def lib_thresholds(row, n):
    """Thresholds T[0..n-1] of an Ising row: 2^32 where the 'always' bit is set."""
    always = int(row[15])
    return [TWO32 if (always >> k) & 1 else int(row[k]) for k in range(n)]


@pytest.mark.parametrize("beta", BETAS)
def test_ising_metropolis_and_heat_bath_tables(beta):
    assert lib_thresholds(B.threshold_row(B.ISING, B.METROPOLIS, beta), 3) == \
        [int(t) for t in oracle.tables_metropolis(beta)]
    assert lib_thresholds(B.threshold_row(B.ISING, B.HEATBATH, beta), 7) == \
        [int(t) for t in oracle.tables_heatbath(beta)]


@pytest.mark.parametrize("beta", BETAS)
def test_potts_weights(beta):
    W = [int(w) for w in oracle.tables_potts(beta)]
    for model in (B.POTTS, B.GPOTTS, B.GPOTTS4):
        row = B.threshold_row(model, B.HEATBATH, beta)
        assert [int(v) for v in row[:13]] == W
        assert not row[13:].any()


def test_the_documented_values_at_the_benchmark_temperatures():
    # thresholds at T = 1.1 and weights at T = 0.9 as printed in the design notes
    assert lib_thresholds(B.threshold_row(B.ISING, B.METROPOLIS, 1 / 1.1), 3) == \
        [78560, 2981635, 113163715]
    assert lib_thresholds(B.threshold_row(B.ISING, B.HEATBATH, 1 / 1.1), 7) == \
        [78558, 2979566, 110258623, 2147483648, 4184708672, 4291987729, 4294888737]
    assert [int(v) for v in B.threshold_row(B.POTTS, B.HEATBATH, 1 / 0.9)[:13]] == \
        [268435456, 88367069, 29089819, 9576164, 3152406, 1037750, 341620, 112458, 37020,
         12186, 4011, 1320, 434]


def test_pt_factors():
    temps = inputs.linear_temperatures(32, 0.7, 1.6)
    pairs = [(1 / temps[i], 1 / temps[i + 1]) for i in range(31)]
    pairs += [(0.5, 0.5), (1.0, 0.0), (0.3, 2.0), (3.0, 1e-3)]
    for bi, bn in pairs:
        F, sgn = B.pt_factors(bi, bn)
        assert [int(f) for f in F] == [int(f) for f in oracle.tables_pt(bi, bn)]
        assert sgn == int(np.sign(bi - bn))


# ---------------------------------------------------------------------------
# Ising-like models (Eq. 2): the library tabulates one threshold per site
# class (k, phi), k = n_empty + 2 n_good in 0..12; the oracle evaluates the
# threshold of each site update from the local field.  For every class a
# site is built whose neighbourhood has that class, and the oracle's
# threshold is measured as the number of r in [0, 2^32) that move the site.
# ---------------------------------------------------------------------------

L4 = 4
SITE = 0  # (0, 0, 0)
# neighbours of site 0 on L = 4 in the order x+, x-, y+, y-, z+, z-
NBS = [1, 3, 4, 12, 16, 48]


def class_instance(algo, k, phi):
    n_good, n_empty = k // 2, k % 2
    N = L4 ** 3
    D = np.ones((5, N), np.int8)
    s = np.ones(N, np.int8)
    for j, nb in enumerate(NBS):
        if j < n_empty:
            D[3, nb] = 0
        elif j < n_empty + n_good:
            s[nb] = 1   # J = +1 and s_i = +1: the bond term is +1
        else:
            s[nb] = -1
    # Metropolis: phi = [s_i f_i = -1] (s_i = +1); heat bath: phi = [f_i = -1]
    D[4, SITE] = -1 if phi else 1
    return D, s


def oracle_threshold(algo, D, s, field, beta):
    lo, hi = 0, TWO32
    while lo < hi:
        mid = (lo + hi) // 2
        u = s.copy()
        oracle.isinggen_update_site(L4, algo, u, D, field, beta, SITE, mid)
        hit = (u[SITE] != s[SITE]) if algo == oracle.METROPOLIS else (u[SITE] == 1)
        lo, hi = (mid + 1, hi) if hit else (lo, mid)
    return lo


@pytest.mark.parametrize("algo", [B.METROPOLIS, B.HEATBATH])
@pytest.mark.parametrize("field", [0.0, 0.3, 1.5])
def test_ising_like_class_thresholds(algo, field):
    for beta in (0.0, 1e-3, 0.3, 1 / 1.1, 2.0, 20.0):
        row = B.threshold_row(B.ISING_GEN, algo, beta, field)
        for phi in (0, 1):
            lim = int(row[13 + 16 * phi])
            for k in range(13):
                certain = k < lim if algo == B.METROPOLIS else k >= lim
                lib = TWO32 if certain else int(row[k + 16 * phi])
                if certain:
                    assert row[k + 16 * phi] == 0
                D, s = class_instance(algo, k, phi)
                assert lib == oracle_threshold(algo, D, s, field, beta), (beta, phi, k)


def test_invalid_table_requests_are_rejected():
    for args, code in (((7, B.METROPOLIS, 1.0, 0.0), B.SG_E_INVALID),
                       ((B.ISING, 3, 1.0, 0.0), B.SG_E_INVALID),
                       ((B.ISING, B.METROPOLIS, -1.0, 0.0), B.SG_E_INVALID),
                       ((B.ISING, B.METROPOLIS, float("nan"), 0.0), B.SG_E_INVALID),
                       ((B.POTTS, B.METROPOLIS, 1.0, 0.0), B.SG_E_UNSUPPORTED),
                       ((B.ISING_GEN, B.METROPOLIS, 1.0, -1.0), B.SG_E_INVALID)):
        with pytest.raises(B.SgError) as e:
            B.threshold_row(*args)
        assert e.value.code == code
    with pytest.raises(B.SgError):
        B.pt_factors(float("inf"), 1.0)
