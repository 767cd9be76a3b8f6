"""Pins of the oracle's exact Bernoulli thresholds.

T_inf[k] = floor(2^32 * (1 - (1 - beta)^k)) and T_rec = floor(2^32 * gamma)
are the round-down uint32 thresholds of the grid SIR (infection probability
1 - (1 - beta)^k for k infected neighbours, a reformulation of the
contact-driven infection of Sec. 5.1.2).  The oracle computes them with
``fractions.Fraction``; here they are checked against arbitrary-precision
floating point (mpmath, a different route), against expanded closed forms for
small k, and against the properties any correct table must have.
"""
from fractions import Fraction

import pytest

from oracle import thresholds as TH

mpmath = pytest.importorskip("mpmath")

SWEEP = [(15 + 19 * j, 1500) for j in range(16)]   # 16 linear values 1/100 .. 1/5
CONFIG_BETAS = [(1, 20)] + SWEEP + [(1, 3), (999, 1000), (1, 1000), (7, 9)]


def _mp_threshold(num, den, k):
    """floor(2^32 (1 - (1 - num/den)^k)) in high-precision floating point,
    refusing cases that land too close to an integer to decide."""
    with mpmath.workdps(80):
        p = 1 - (1 - mpmath.mpf(num) / den) ** k
        v = p * mpmath.mpf(2) ** 32
        f = mpmath.floor(v)
        assert v - f > mpmath.mpf(10) ** -40 or v == f
        return int(f)


@pytest.mark.parametrize("beta", CONFIG_BETAS)
def test_table_matches_mpmath(beta):
    table, k_sat = TH.infection_table(*beta)
    assert len(table) == k_sat + 1
    ks = sorted(set(list(range(0, min(k_sat, 40) + 1)) +
                    list(range(0, k_sat + 1, max(1, k_sat // 50))) + [k_sat]))
    for k in ks:
        assert table[k] == _mp_threshold(*beta, k), (beta, k)


@pytest.mark.parametrize("beta", CONFIG_BETAS)
def test_table_shape(beta):
    table, k_sat = TH.infection_table(*beta)
    assert table[0] == 0
    assert all(a <= b for a, b in zip(table, table[1:]))
    assert table[-1] == 2 ** 32 - 1
    assert all(t < 2 ** 32 - 1 for t in table[:-1])
    # k_sat is where (1 - beta)^k first drops to 2^-32 or below
    with mpmath.workdps(60):
        miss = lambda k: (1 - mpmath.mpf(beta[0]) / beta[1]) ** k * mpmath.mpf(2) ** 32
        assert miss(k_sat) <= 1 and miss(k_sat - 1) > 1


@pytest.mark.parametrize("beta", CONFIG_BETAS)
def test_small_k_closed_forms(beta):
    n, d = beta
    table, _ = TH.infection_table(n, d)
    # k = 1: p = beta
    assert table[1] == (n << 32) // d
    # k = 2: p = 2 beta - beta^2 = n (2d - n) / d^2
    if len(table) > 2:
        assert table[2] == ((n * (2 * d - n)) << 32) // (d * d)
    # k = 3: p = 3b - 3b^2 + b^3 = n (3d^2 - 3dn + n^2) / d^3
    if len(table) > 3:
        assert table[3] == ((n * (3 * d * d - 3 * d * n + n * n)) << 32) // d ** 3


@pytest.mark.parametrize("beta", [(1, 20)] + SWEEP)
def test_error_bound(beta):
    """|T_k / 2^32 - p_k| < 2^-32 for every entry."""
    table, k_sat = TH.infection_table(*beta)
    with mpmath.workdps(60):
        for k in range(0, k_sat + 1, max(1, k_sat // 200)):
            p = 1 - (1 - mpmath.mpf(beta[0]) / beta[1]) ** k
            err = abs(mpmath.mpf(table[k]) / 2 ** 32 - p)
            assert err < mpmath.mpf(2) ** -32


def test_beta_zero_and_recovery():
    assert TH.infection_table(0, 7) == ([0], 0)
    assert TH.recovery_threshold(0, 5) == 0
    assert TH.recovery_threshold(1, 100) == 42949672      # floor(2^32 / 100)
    assert TH.recovery_threshold(1, 2) == 2 ** 31
    for g in [(1, 3), (2, 3), (99, 100), (1, 7)]:
        assert TH.recovery_threshold(*g) == _mp_threshold(*g, 1)


def test_rejects_invalid():
    for bad in [(1, 1), (2, 1), (-1, 5), (1, 0)]:
        with pytest.raises(ValueError):
            TH.infection_table(*bad)
        with pytest.raises(ValueError):
            TH.recovery_threshold(*bad)


def test_sweep_saturation_points():
    """k_sat shrinks as beta grows, and beta = 1/100 needs the longest table."""
    ks = [TH.infection_table(*b)[1] for b in SWEEP]
    assert all(a > b for a, b in zip(ks, ks[1:]))
    assert Fraction(*SWEEP[0]) == Fraction(1, 100) and Fraction(*SWEEP[-1]) == Fraction(1, 5)
    assert max(ks) < 4096
