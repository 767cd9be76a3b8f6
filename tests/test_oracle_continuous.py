"""Pins of the oracle's continuous-space models (the paper's benchmark
models of Sec. 5.1.2: the clamped random walk and the SIR with contacts
within radius 5, probability 0.1 per contact, recovery after 14 days, five
initially infected), against the brute force's own Philox and numpy float32
scalar arithmetic with a pairwise contact loop, and against the invariants
of Sec. 5.1.3."""
import numpy as np
import pytest


@pytest.mark.parametrize("model,n,W,r,steps", [("walk", 50, 10.0, 1.0, 30), ("sir", 60, 12.0, 2.5, 25),
                                               ("sir", 40, 3.0, 5.0, 18), ("sir", 1, 5.0, 1.0, 5)])
def test_continuous_models_match_brute_force(oracle_mod, model, n, W, r, steps):
    from oracle import brute
    m = oracle_mod.RANDOM_WALK if model == "walk" else oracle_mod.SIR
    o = oracle_mod.ContRun(m, n, W=W, r=r, seed=2, stream=7, p=(1, 3), recover=6,
                           initial_infected=min(5, n)).step(steps)
    xs, ys, st, days = brute.cont_run(model, n, W, r, 2, 7, steps, p=(1, 3), recover=6,
                                      i0=min(5, n))
    assert np.array_equal(o.x, np.array(xs, np.float32))
    assert np.array_equal(o.y, np.array(ys, np.float32))
    if model == "sir":
        assert o.s.tolist() == st and o.days.tolist() == days


def test_paper_sir_invariants_and_recovery_after_14_days(oracle_mod):
    n = 2000
    o = oracle_mod.ContRun(oracle_mod.SIR, n, seed=0, stream=0)
    assert (o.s == 1).sum() == 5                          # five initially infected
    became_i = {a: 0 for a in range(5)}
    became_r = {}
    for t in range(60):
        before = o.s.copy()
        o.step(1)
        assert ((o.s == 0) | (o.s == 1) | (o.s == 2)).all() and len(o.s) == n
        assert (o.x >= 0).all() and (o.x <= 100).all() and (o.y >= 0).all() and (o.y <= 100).all()
        for a in np.flatnonzero((before == 0) & (o.s == 1)):
            became_i[int(a)] = t + 1
        for a in np.flatnonzero((before == 1) & (o.s == 2)):
            became_r[int(a)] = t + 1
        assert not ((before == 2) & (o.s != 2)).any()      # R is absorbing
        assert not ((before == 0) & (o.s == 2)).any()      # no S -> R in one step
    assert len(became_r) > 5                               # the epidemic spread and recovered
    for a, tr in became_r.items():
        assert tr - became_i[a] == 14


def test_continuous_special_cases(oracle_mod):
    # no transmission: only the initial five are ever infected
    o = oracle_mod.ContRun(oracle_mod.SIR, 500, W=10.0, seed=1, stream=1, p=(0, 1)).step(10)
    assert (o.s != 0).sum() == 5
    # a world of side 0 keeps everyone at the origin
    o = oracle_mod.ContRun(oracle_mod.RANDOM_WALK, 100, W=0.0, seed=1, stream=1).step(5)
    assert (o.x == 0).all() and (o.y == 0).all()
    # a wide world: no clamping in 10 steps from the middle, so each step
    # moves every coordinate by less than 1
    o = oracle_mod.ContRun(oracle_mod.RANDOM_WALK, 1000, W=1e4, seed=3, stream=1)
    x0 = o.x.copy()
    o.step(1)
    assert (np.abs(o.x - x0) <= 1.0).all() and (o.x != x0).any()
