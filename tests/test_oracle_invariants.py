"""Pins of the oracle's invariant checks (the correctness checks of Sec. 5.1.3:
conserved wealth, positions on the grid, S + I + R = N) on rows that break
them, and of the digest's finaliser.

Every expected count here is fixed by construction: a population of valid
rows with a known number of rows of each kind planted at known places, so a
wrong bound ('>' for '>='), an uncounted state code or a row counted twice
fails a test.  The digest's finaliser is pinned to SplitMix64's published
outputs (Steele, Lea and Flood, OOPSLA'14).
"""
import numpy as np
import pytest


def _planted_grid(L, n, rng):
    x = rng.integers(0, L, n).astype(np.int32)
    y = rng.integers(0, L, n).astype(np.int32)
    # valid edge values at known rows
    x[0], y[0] = 0, 0
    x[1], y[1] = L - 1, L - 1
    return x, y


@pytest.mark.parametrize("L", [1, 2, 3, 1000])
def test_positions_out_of_grid_are_counted_once_per_row(oracle_mod, L):
    rng = np.random.default_rng(L)
    n = 3000
    x, y = _planted_grid(L, n, rng)
    assert oracle_mod.invariants(n, L, x=x, y=y)["out_of_bounds"] == 0
    # one bad coordinate per row: x = L, x = -1, y = L, y = -1, far outside
    planted = {10: ("x", L), 11: ("x", -1), 12: ("y", L), 13: ("y", -1),
               14: ("x", 2**31 - 1), 15: ("y", -(2**31))}
    for row, (col, v) in planted.items():
        (x if col == "x" else y)[row] = v
    # both coordinates bad in one row: still one row
    x[20], y[20] = L, -1
    assert oracle_mod.invariants(n, L, x=x, y=y)["out_of_bounds"] == len(planted) + 1


def test_wealth_below_zero_is_counted_and_min_reported(oracle_mod):
    n = 2000
    w = np.ones(n, dtype=np.int32)
    w[5] = 0                         # zero wealth is valid
    w[7], w[8], w[9] = -1, -5, -(2**31)
    w[10] = 2**31 - 1
    inv = oracle_mod.invariants(n, 0, w=w)
    assert inv["out_of_bounds"] == 3
    assert inv["wealth_min"] == -(2**31)
    # sum by construction: n - 1 ones, minus the rows overwritten, plus the planted values
    assert inv["wealth_sum"] == (n - 5) * 1 + 0 - 1 - 5 - 2**31 + (2**31 - 1)
    w2 = np.full(n, 3, dtype=np.int32)
    w2[0] = -1
    inv = oracle_mod.invariants(n, 0, w=w2)
    assert (inv["wealth_min"], inv["out_of_bounds"], inv["wealth_sum"]) == (-1, 1, 3 * (n - 1) - 1)


def test_state_codes_above_two_are_counted_not_classified(oracle_mod):
    n, L = 4000, 50
    rng = np.random.default_rng(3)
    x, y = _planted_grid(L, n, rng)
    s = np.zeros(n, dtype=np.uint8)
    s[100:400] = 1                   # 300 infected
    s[400:450] = 2                   # 50 recovered
    s[450], s[451], s[452] = 3, 4, 255
    inv = oracle_mod.invariants(n, L, x=x, y=y, s=s)
    assert (inv["n_s"], inv["n_i"], inv["n_r"]) == (n - 353, 300, 50)
    assert inv["out_of_bounds"] == 3
    assert inv["n_s"] + inv["n_i"] + inv["n_r"] + inv["out_of_bounds"] == n
    # a row with a bad state and a bad position counts once
    x[450] = L
    assert oracle_mod.invariants(n, L, x=x, y=y, s=s)["out_of_bounds"] == 3
    x[451] = -1                       # already bad by its state
    y[500] = L                        # a susceptible row off the grid
    inv = oracle_mod.invariants(n, L, x=x, y=y, s=s)
    assert inv["out_of_bounds"] == 4 and inv["n_s"] == n - 353


def test_valid_runs_have_no_bad_rows(oracle_mod):
    for model in (0, 1, 2):
        r = oracle_mod.OracleRun(model, 777, 9, seed=2, stream=5).step(20)
        assert r.invariants()["out_of_bounds"] == 0


def test_finaliser_matches_published_splitmix64_outputs(oracle_mod):
    # SplitMix64 seeded with 0: outputs k = 1, 2, 3 are the finaliser of
    # k * 0x9E3779B97F4A7C15 (mod 2^64)
    gamma = 0x9E3779B97F4A7C15
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = [oracle_mod.fmix64((k * gamma) & (2**64 - 1)) for k in (1, 2, 3)]
    assert got == want
    assert oracle_mod.fmix64(0) == 0


def test_digest_of_one_row_is_the_chained_finaliser(oracle_mod):
    # one agent (id 0) with one int32 column holding v: fmix64(fmix64(0) ^ (1 << 32 | v)),
    # and fmix64(0) = 0
    for v in (0, 1, 123456789):
        col = np.array([v], dtype=np.int32)
        assert oracle_mod.digest([col]) == oracle_mod.fmix64((1 << 32) | v)
