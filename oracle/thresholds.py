"""Exact uint32 Bernoulli thresholds for the grid SIR (TEST INFRASTRUCTURE).

A Bernoulli(p) trial succeeds iff a uniform 32-bit word u satisfies u < T with
T = floor(p * 2^32), computed here in exact rational arithmetic
(``fractions.Fraction``).  The infection probability for a susceptible agent
with k infected agents in its neighbourhood is 1 - (1 - beta)^k (the grid
reformulation of the contact-driven infection of Sec. 5.1.2, with one
independent trial per infected neighbour); recovery has probability gamma per
step.  beta and gamma are exact rationals num/den with 0 <= num < den, so every
threshold is below 2^32.
"""
from fractions import Fraction

TWO32 = 1 << 32
T_MAX = TWO32 - 1


def bernoulli_threshold(p: Fraction) -> int:
    """floor(p * 2^32) for a rational 0 <= p < 1."""
    if not (0 <= p < 1):
        raise ValueError("probability must lie in [0, 1)")
    return (p.numerator * TWO32) // p.denominator


def infection_table(beta_num: int, beta_den: int):
    """Return (T_inf, k_sat) with T_inf[k] = floor(2^32 (1 - (1-beta)^k)) for
    k = 0..k_sat, where k_sat is the first k at which the threshold stops
    changing: for beta > 0 the first k with T = 2^32 - 1, for beta = 0 it is 0.
    Every k > k_sat uses T_inf[k_sat]."""
    if beta_den <= 0 or not (0 <= beta_num < beta_den):
        raise ValueError("need 0 <= beta_num < beta_den")
    beta = Fraction(beta_num, beta_den)
    if beta == 0:
        return [0], 0
    keep = 1 - beta          # probability that one infected neighbour fails
    miss = Fraction(1)       # (1 - beta)^k
    table = []
    k = 0
    while True:
        t = bernoulli_threshold(1 - miss)
        table.append(t)
        if t == T_MAX:
            return table, k
        k += 1
        miss *= keep


def recovery_threshold(gamma_num: int, gamma_den: int) -> int:
    if gamma_den <= 0 or not (0 <= gamma_num < gamma_den):
        raise ValueError("need 0 <= gamma_num < gamma_den")
    return bernoulli_threshold(Fraction(gamma_num, gamma_den))
