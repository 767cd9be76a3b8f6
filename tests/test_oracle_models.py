"""Pins of the oracle's model steps: wealth transfer, torus random walk, grid
SIR (Sec. 5.1.2 reformulated on a torus grid; synchronous semantics, Sec. 3.4;
invariants, Sec. 5.1.3).

Each pin is independent of the oracle's own code: the pure-Python brute force
(own Philox, O(N^2) neighbour search), numpy's ``add.at`` (the scatter-add the
paper's view API is built on, Sec. 3.1.1), exhaustive enumeration, closed
forms and invariants.
"""
import itertools
import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import brute


# ------------------------------------------------------------------ wealth

def _sequential_transfers(w, recip):
    """Move one unit at a time, donors fixed by the snapshot (a different
    algorithm from the oracle's column update)."""
    out = list(w)
    donors = [a for a in range(len(w)) if w[a] > 0]
    for a in donors:
        out[a] -= 1
        out[recip[a]] += 1
    return out


def test_wealth_apply_exhaustive_small(oracle_mod):
    """Every wealth state in {0,1,2}^N and every recipient tuple, N <= 3."""
    for n in (1, 2, 3):
        for w in itertools.product(range(3), repeat=n):
            for recip in itertools.product(range(n), repeat=n):
                got = oracle_mod.wealth_apply(np.array(w), np.array(recip))
                assert list(got) == _sequential_transfers(w, recip)
                assert got.sum() == sum(w)


def test_wealth_apply_matches_numpy_add_at(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(200):
        n = int(rng.integers(1, 300))
        w = rng.integers(0, 4, n).astype(np.int32)
        recip = rng.integers(0, n, n).astype(np.uint32)
        donors = w > 0
        want = w.copy()
        want[donors] -= 1
        np.add.at(want, recip[donors], 1)
        assert (oracle_mod.wealth_apply(w, recip) == want).all()


def test_wealth_hammer_same_recipient(oracle_mod):
    """All donors choose one recipient: no lost updates."""
    n, target = 257, 100
    w = np.ones(n, dtype=np.int32)
    w[::3] = 0
    got = oracle_mod.wealth_apply(w, np.full(n, target))
    donors = int((w > 0).sum())
    assert got[target] == w[target] + donors - int(w[target] > 0)
    others = np.arange(n) != target
    assert (got[others] == 0).all()


@pytest.mark.parametrize("n,steps,w0,seed,stream", [(1, 5, 1, 0, 0), (2, 9, 1, 3, 1),
                                                    (10, 20, 2, 1, 2), (37, 15, 1, 5, 9),
                                                    (64, 12, 3, 0, 7)])
def test_wealth_oracle_matches_brute(oracle_mod, n, steps, w0, seed, stream):
    r = oracle_mod.OracleRun(oracle_mod.WEALTH, n, seed=seed, stream=stream, wealth_init=w0)
    r.step(steps)
    assert list(r.w) == brute.wealth_run(n, w0, seed, stream, steps)


def test_wealth_recipient_mapping(oracle_mod):
    """recipient = floor(U * N / 2^64), U = (word0 << 32) | word1."""
    for n in (1, 2, 3, 1000, 10 ** 7, 2 ** 31 - 1):
        for t, a in [(0, 0), (5, 17), (99, 123456)]:
            hi = oracle_mod.word(0, 0, 3, 2, t, a, 0)
            lo = oracle_mod.word(0, 0, 3, 2, t, a, 1)
            r = oracle_mod.recipient(n, 0, 0, t, a)
            assert r == ((hi << 32 | lo) * n) >> 64 and 0 <= r < n


@settings(max_examples=40, deadline=None)
@given(n=st.integers(1, 400), seed=st.integers(0, 2 ** 32 - 1),
       stream=st.integers(0, 2 ** 32 - 1), w0=st.integers(0, 5), steps=st.integers(1, 30))
def test_wealth_conservation(oracle_mod, n, seed, stream, w0, steps):
    r = oracle_mod.OracleRun(oracle_mod.WEALTH, n, seed=seed, stream=stream, wealth_init=w0)
    for _ in range(steps):
        r.step(1)
        inv = r.invariants()
        assert inv["wealth_sum"] == n * w0 and inv["wealth_min"] >= 0
        assert inv["out_of_bounds"] == 0


def test_wealth_single_agent_is_fixed(oracle_mod):
    r = oracle_mod.OracleRun(oracle_mod.WEALTH, 1, seed=4, wealth_init=3).step(50)
    assert list(r.w) == [3]


# ------------------------------------------------------------------ random walk

@pytest.mark.parametrize("n,L,steps,seed,stream", [(1, 1, 5, 0, 0), (5, 2, 9, 1, 0),
                                                   (30, 3, 12, 2, 3), (50, 7, 20, 9, 1),
                                                   (64, 1000, 25, 0, 0)])
def test_walk_oracle_matches_brute(oracle_mod, n, L, steps, seed, stream):
    r = oracle_mod.OracleRun(oracle_mod.RANDOM_WALK, n, L, seed=seed, stream=stream).step(steps)
    x, y = brute.walk_run(n, L, seed, stream, steps)
    assert list(r.x) == x and list(r.y) == y


def test_walk_closed_form_displacement(oracle_mod):
    """x_T - x_0 - sum(dx_t) == 0 (mod L) for every agent, with the unwrapped
    displacement summed from the brute-force draws."""
    n, L, T, seed, stream = 200, 11, 40, 5, 6
    r0 = oracle_mod.OracleRun(oracle_mod.RANDOM_WALK, n, L, seed=seed, stream=stream)
    x0, y0 = r0.x.copy(), r0.y.copy()
    r0.step(T)
    for a in range(n):
        dx = dy = 0
        for t in range(T):
            mx, my = brute.MOVES[brute.draw(seed, stream, "move", t, a, 0) >> 29]
            dx, dy = dx + mx, dy + my
        assert (r0.x[a] - x0[a] - dx) % L == 0 and (r0.y[a] - y0[a] - dy) % L == 0


def test_walk_agents_replay_matches_full_run(oracle_mod):
    n, L, T = 3000, 97, 30
    r = oracle_mod.OracleRun(oracle_mod.RANDOM_WALK, n, L, seed=1, stream=2).step(T)
    ids = np.array([0, 1, 2, 3, 4, 1000, 2999, 1777], dtype=np.uint32)
    x, y = oracle_mod.walk_agents(ids, L, 1, 2, T)
    assert (x == r.x[ids]).all() and (y == r.y[ids]).all()


def test_walk_bounds_and_degenerate_grids(oracle_mod):
    r = oracle_mod.OracleRun(oracle_mod.RANDOM_WALK, 100, 1, seed=3).step(10)
    assert (r.x == 0).all() and (r.y == 0).all()
    for L in (2, 3, 1000):
        r = oracle_mod.OracleRun(oracle_mod.RANDOM_WALK, 500, L, seed=3).step(10)
        assert r.invariants()["out_of_bounds"] == 0
        assert r.x.min() >= 0 and r.x.max() < L


def test_walk_direction_table():
    """The 8 Moore moves in lexicographic (dx, dy) order, (0,0) excluded."""
    assert brute.MOVES == [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]


def test_init_positions_uniform_mapping(oracle_mod):
    n, L = 64, 1000
    r = oracle_mod.OracleRun(oracle_mod.RANDOM_WALK, n, L, seed=2, stream=8)
    for a in range(n):
        assert r.x[a] == (oracle_mod.word(2, 8, 0, 2, 0, a, 0) * L) >> 32
        assert r.y[a] == (oracle_mod.word(2, 8, 0, 2, 0, a, 1) * L) >> 32


# ------------------------------------------------------------------ SIR

@pytest.mark.parametrize("L", [1, 2, 3, 4, 5])
def test_neighbour_count_matches_pairwise_brute(oracle_mod, L):
    rng = random.Random(L)
    for _ in range(30):
        n = rng.randrange(1, 40)
        agents = [{"x": rng.randrange(L), "y": rng.randrange(L)} for _ in range(n)]
        states = [rng.randrange(3) for _ in range(n)]
        C = np.zeros((L, L), dtype=np.uint32)
        for ag, s in zip(agents, states):
            if s == 1:
                C[ag["y"], ag["x"]] += 1
        for a in range(n):
            k = oracle_mod.neighbour_infected(L, C, agents[a]["x"], agents[a]["y"])
            assert k == brute.sir_infected_neighbours(agents, states, a, L)


def test_neighbour_count_dedups_small_torus(oracle_mod):
    """On L < 3 the wrapped 3x3 block covers the whole grid exactly once."""
    for L in (1, 2):
        C = np.arange(1, L * L + 1, dtype=np.uint32)
        for cx in range(L):
            for cy in range(L):
                assert oracle_mod.neighbour_infected(L, C, cx, cy) == C.sum()
    C = np.zeros(9, dtype=np.uint32)
    C[4] = 5
    assert oracle_mod.neighbour_infected(3, C, 0, 0) == 5  # all 9 cells distinct


@pytest.mark.parametrize("n,L,steps,beta,gamma,seed,stream,i0", [
    (1, 1, 5, (1, 20), (1, 100), 0, 0, None),
    (6, 1, 8, (1, 2), (1, 3), 1, 0, 2),
    (9, 2, 10, (1, 3), (1, 5), 2, 1, 3),
    (25, 3, 12, (1, 4), (1, 10), 3, 2, 4),
    (40, 5, 15, (1, 20), (1, 100), 4, 3, 5),
    (60, 8, 20, (34, 1500), (1, 100), 5, 11, 7),
    (80, 9, 10, (300, 1500), (1, 100), 0, 255, None),
])
def test_sir_oracle_matches_brute(oracle_mod, n, L, steps, beta, gamma, seed, stream, i0):
    r = oracle_mod.OracleRun(oracle_mod.SIR, n, L, seed=seed, stream=stream, beta=beta,
                             gamma=gamma, initial_infected=i0 or 0).step(steps)
    x, y, s = brute.sir_run(n, L, seed, stream, steps, beta, gamma, i0)
    assert list(r.x) == x and list(r.y) == y and list(r.s) == s


def test_sir_invariants_over_a_run(oracle_mod):
    n, L = 3000, 40
    r = oracle_mod.OracleRun(oracle_mod.SIR, n, L, seed=1, beta=(1, 5), gamma=(1, 20))
    i0 = max(1, (n + 500) // 1000)
    inv = r.invariants()
    assert inv["n_i"] == i0 and inv["n_s"] == n - i0 and inv["n_r"] == 0
    prev_s, prev = r.s.copy(), inv
    for _ in range(60):
        r.step(1)
        inv = r.invariants()
        assert inv["n_s"] + inv["n_i"] + inv["n_r"] == n
        assert inv["out_of_bounds"] == 0
        assert inv["n_s"] <= prev["n_s"] and inv["n_r"] >= prev["n_r"]
        assert (r.s >= prev_s).all()                      # S -> I -> R only
        assert ((r.s - prev_s) <= 1).all()                # one transition per step
        prev_s, prev = r.s.copy(), inv
    assert inv["n_r"] > 0 and inv["n_s"] < n - i0


def test_sir_without_transmission_is_a_random_walk(oracle_mod):
    """beta = gamma = 0: positions equal the random walk with the same key,
    S is constant and nobody recovers."""
    n, L, T = 500, 23, 30
    sir = oracle_mod.OracleRun(oracle_mod.SIR, n, L, seed=7, stream=3, beta=(0, 1), gamma=(0, 1)).step(T)
    rw = oracle_mod.OracleRun(oracle_mod.RANDOM_WALK, n, L, seed=7, stream=3).step(T)
    assert (sir.x == rw.x).all() and (sir.y == rw.y).all()
    inv = sir.invariants()
    assert inv["n_s"] == n - 1 and inv["n_r"] == 0 and inv["n_i"] == 1


def test_sir_no_infected_neighbours_no_infection(oracle_mod):
    """An isolated infected agent on a huge grid never infects anyone."""
    r = oracle_mod.OracleRun(oracle_mod.SIR, 2, 2000, seed=0, beta=(999, 1000), gamma=(0, 1))
    far = abs(int(r.x[0]) - int(r.x[1])) > 50 or abs(int(r.y[0]) - int(r.y[1])) > 50
    assert far
    r.step(20)
    assert list(r.s) == [1, 0]


def test_sir_initial_infected_count(oracle_mod):
    for n, want in [(1, 1), (499, 1), (1000, 1), (1499, 1), (1500, 2), (10 ** 6, 1000)]:
        assert oracle_mod.default_initial_infected(n) == want
    r = oracle_mod.OracleRun(oracle_mod.SIR, 5000, 70, initial_infected=17)
    assert r.invariants()["n_i"] == 17 and (r.s[:17] == 1).all() and (r.s[17:] == 0).all()


def test_grid_side_rounding(oracle_mod):
    import math
    for n in list(range(1, 3000)) + [10 ** 6, 10 ** 7, 2 ** 27, 2 ** 31 - 1]:
        L = oracle_mod.grid_side(n)
        assert abs(L - math.sqrt(n)) <= 0.5 + 1e-12
        # halves never occur for integers: check against exact comparison
        assert (2 * L - 1) ** 2 < 4 * n <= (2 * L + 1) ** 2 or n == 0
    assert [oracle_mod.grid_side(n) for n in (1000, 1500, 10 ** 7)] == [32, 39, 3162]


# ------------------------------------------------------------------ common

@pytest.mark.parametrize("model", [0, 1, 2])
def test_chunking_invariance(oracle_mod, model):
    a = oracle_mod.OracleRun(model, 700, 30, seed=2, stream=1).step(7).step(1).step(12)
    b = oracle_mod.OracleRun(model, 700, 30, seed=2, stream=1).step(20)
    assert a.digest() == b.digest()
    for ca, cb in zip(a.columns(), b.columns()):
        assert (ca == cb).all()


@pytest.mark.parametrize("model", [0, 1, 2])
def test_seed_and_stream_change_results(oracle_mod, model):
    base = oracle_mod.OracleRun(model, 500, 25, seed=0, stream=0).step(10).digest()
    assert base == oracle_mod.OracleRun(model, 500, 25, seed=0, stream=0).step(10).digest()
    assert base != oracle_mod.OracleRun(model, 500, 25, seed=1, stream=0).step(10).digest()
    assert base != oracle_mod.OracleRun(model, 500, 25, seed=0, stream=1).step(10).digest()


def _np_fmix(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def test_digest_matches_numpy_formulation(oracle_mod):
    rng = np.random.default_rng(0)
    n = 5000
    x = rng.integers(0, 1000, n).astype(np.int32)
    y = rng.integers(0, 1000, n).astype(np.int32)
    s = rng.integers(0, 3, n).astype(np.uint8)
    with np.errstate(over="ignore"):
        h = _np_fmix(np.arange(n, dtype=np.uint64))
        for j, col in enumerate([x, y, s]):
            v = col.astype(np.int64).astype(np.uint64) & np.uint64(0xFFFFFFFF)
            h = _np_fmix(h ^ ((np.uint64(j + 1) << np.uint64(32)) | v))
        want = int(h.sum(dtype=np.uint64))
    assert oracle_mod.digest([x, y, s]) == want
    # order-free over agents only through the id: a swap of rows changes it
    x2 = x.copy(); x2[[0, 1]] = x2[[1, 0]]
    assert oracle_mod.digest([x2, y, s]) != want or x[0] == x[1]
