"""Pins of the oracle's buffered write log (the pending-writes flush of
Sec. 3.2.1) and of asynchronous (sequential) update semantics (Sec. 3.4) for
the wealth model.

  * write log: a Python dict filled in log order (the paper's pending-writes
    dictionary: the last write to a key stays), then applied;
  * acting order: Python's sorted() over (ORDER word, id) with the brute
    force's own Philox;
  * async wealth: the brute force's sequential simulation on tiny
    populations; wealth conserved and never negative; and with every agent
    holding at least one unit, every agent gives in either semantics, so the
    asynchronous step equals the synchronous one.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_write_log_last_write_wins(oracle_mod, dtype):
    rng = np.random.default_rng(1)
    n, m = 200, 3000
    col = rng.integers(-50, 50, n).astype(dtype)
    ids = rng.integers(0, n + 10, m).astype(np.uint32)
    vals = rng.integers(-10**6, 10**6, m).astype(dtype)
    pending = {}
    for i, v in zip(ids.tolist(), vals.tolist()):
        if i < n:
            pending[i] = v
    want = col.copy()
    for i, v in pending.items():
        want[i] = v
    assert np.array_equal(oracle_mod.write_log(col, ids, vals), want)
    # float32 bits kept: -0.0 and a subnormal survive the flush
    if dtype == np.float32:
        got = oracle_mod.write_log(np.ones(2, np.float32), [0, 1],
                                   np.array([-0.0, 1e-42], np.float32))
        assert np.signbit(got[0]) and got[1] == np.float32(1e-42)


def test_write_log_empty_and_out_of_range(oracle_mod):
    col = np.arange(5, dtype=np.int32)
    assert np.array_equal(oracle_mod.write_log(col, [], []), col)
    assert np.array_equal(oracle_mod.write_log(col, [5, 99], [1, 2]), col)


@pytest.mark.parametrize("n,t", [(1, 0), (7, 3), (50, 11)])
def test_async_order_is_sorted_order_words(oracle_mod, n, t):
    from oracle import brute
    want = sorted(range(n), key=lambda a: (brute.draw(5, 9, "order", t, a, 0), a))
    assert oracle_mod.async_order(n, 5, 9, t).tolist() == want


@pytest.mark.parametrize("n,w0,steps", [(1, 3, 4), (2, 1, 5), (9, 1, 6), (40, 2, 5), (64, 0, 2)])
def test_async_wealth_matches_brute_force(oracle_mod, n, w0, steps):
    from oracle import brute
    w = np.full(n, w0, np.int32)
    w[::3] = 0                                 # some agents start without wealth
    got = oracle_mod.run_wealth_async(w, 2, 7, 3, steps)
    assert got.tolist() == brute.wealth_run_async(w.tolist(), 2, 7, 3, steps)


def test_async_wealth_invariants_and_sync_special_case(oracle_mod):
    n = 5000
    w = np.ones(n, np.int32)
    w[::2] = 3
    for steps in (1, 7):
        got = oracle_mod.run_wealth_async(w, 4, 1, 0, steps)
        assert got.sum() == w.sum() and got.min() >= 0
    # every agent holds a unit at the start of step 0: all give under both
    # semantics, with the same recipients
    sync = oracle_mod.OracleRun(oracle_mod.WEALTH, n, seed=4, stream=1, wealth_init=1).step(1)
    assert np.array_equal(oracle_mod.run_wealth_async(np.ones(n, np.int32), 4, 1, 0, 1), sync.w)
    # later steps differ from the synchronous run (agents at 0 that receive
    # before their turn give under the asynchronous rule)
    a5 = oracle_mod.run_wealth_async(np.ones(n, np.int32), 4, 1, 0, 5)
    s5 = oracle_mod.OracleRun(oracle_mod.WEALTH, n, seed=4, stream=1, wealth_init=1).step(5)
    assert not np.array_equal(a5, s5.w)
