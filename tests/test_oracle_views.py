"""Pins of the oracle's view primitives (the three views of Sec. 3.3 and the
listings of Sec. 3.1.1): full-population and filtered updates v <- a*v + b on
int32 and float32 columns, and the id-indexed scatter-add with duplicates;
and of resuming a run from host columns.

What fixes each expected value, other than the oracle itself:
  * the paper's own listings on populations whose result is known by
    construction (wealth += 10; donors with wealth > 0 give one unit);
  * numpy's add.at, the scatter-add primitive the paper names (int32, and
    float32, where add.at adds in list order with float32 rounding);
  * numpy's int32 array arithmetic (wrap-around modulo 2^32) and the
    composition law of affine maps;
  * mpmath: a*v + b evaluated exactly and rounded once to 24 bits (the fused
    multiply-add), and a case where two roundings give another value;
  * splitting a run: T steps equal t steps, then a run resumed from the
    columns for T - t more.
"""
import numpy as np
import pytest


CMPS = ["<", "<=", "==", "!=", ">=", ">"]


def test_listing_full_view_increment(oracle_mod):
    w = np.ones(1000, dtype=np.int32)
    assert (oracle_mod.view_update(w, 1, 10) == 11).all()


def test_listing_filtered_donors_give_one(oracle_mod):
    w = np.array([0, 1, 2, 0, 5, -3], dtype=np.int32)
    # the predicate reads the column before the update: every donor loses
    # exactly one unit, nobody else changes
    got = oracle_mod.view_update(w, 1, -1, pred=w, cmp=">", thr=0)
    assert got.tolist() == [0, 0, 1, 0, 4, -3]


def test_listing_scatter_add_duplicates_accumulate(oracle_mod):
    w = np.zeros(5, dtype=np.int32)
    got = oracle_mod.scatter_add(w, [4, 1, 4, 4, 0], scalar=1)
    assert got.tolist() == [1, 1, 0, 0, 3]


@pytest.mark.parametrize("seed", range(4))
def test_int32_affine_matches_numpy_wraparound(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    col = rng.integers(-2**31, 2**31, 5000, dtype=np.int64).astype(np.int32)
    a, b = (int(v) for v in rng.integers(-2**31, 2**31, 2))
    with np.errstate(over="ignore"):
        want = col * np.int32(a) + np.int32(b)
    assert np.array_equal(oracle_mod.view_update(col, a, b), want)


def test_int32_affine_special_cases_and_composition(oracle_mod):
    col = np.array([0, 1, -1, 2**31 - 1, -2**31, 12345], dtype=np.int32)
    assert np.array_equal(oracle_mod.view_update(col, 1, 0), col)
    assert (oracle_mod.view_update(col, 0, 77) == 77).all()
    assert oracle_mod.view_update(col, -1, 0).tolist() == [0, -1, 1, -2**31 + 1, -2**31, -12345]
    assert oracle_mod.view_update(col, 1, 1)[3] == -2**31              # wraps
    rng = np.random.default_rng(9)
    for _ in range(20):
        a1, b1, a2, b2 = (int(v) for v in rng.integers(-2**31, 2**31, 4))
        twice = oracle_mod.view_update(oracle_mod.view_update(col, a1, b1), a2, b2)
        a = (a2 * a1) % 2**32
        b = (a2 * b1 + b2) % 2**32
        once = oracle_mod.view_update(col, a - 2**32 if a >= 2**31 else a,
                                      b - 2**32 if b >= 2**31 else b)
        assert np.array_equal(twice, once)


def _fma_exact_f32(a, v, b):
    import mpmath
    with mpmath.workprec(200):
        exact = mpmath.mpf(float(a)) * mpmath.mpf(float(v)) + mpmath.mpf(float(b))
    with mpmath.workprec(24):
        return np.float32(float(+exact))


def test_float32_affine_is_one_rounding(oracle_mod):
    rng = np.random.default_rng(1)
    col = (rng.standard_normal(400) * 1e3).astype(np.float32)
    a, b = np.float32(1.0000001), np.float32(-3.25)
    got = oracle_mod.view_update(col, a, b)
    want = np.array([_fma_exact_f32(a, v, b) for v in col], dtype=np.float32)
    assert np.array_equal(got, want)
    # a case where rounding the product first gives another value: with
    # a = v = 1 + 2^-12 and b = -(1 + 2^-11), a*v + b = 2^-24 exactly, while
    # the rounded product (1 + 2^-11) cancels b to 0
    x = np.float32(1 + 2**-12)
    got = oracle_mod.view_update(np.array([x], dtype=np.float32), x, np.float32(-(1 + 2**-11)))
    assert got[0] == np.float32(2**-24)
    assert np.float32(x * x) + np.float32(-(1 + 2**-11)) == 0      # two roundings differ


@pytest.mark.parametrize("cmp", CMPS)
def test_filtered_update_rows_by_comparison(oracle_mod, cmp):
    # predicate on another column; rows on each side of the threshold and on it
    p = np.array([-5, 2, 3, 3, 4, 100], dtype=np.int32)
    col = np.zeros(6, dtype=np.int32)
    take = {"<": [1, 1, 0, 0, 0, 0], "<=": [1, 1, 1, 1, 0, 0], "==": [0, 0, 1, 1, 0, 0],
            "!=": [1, 1, 0, 0, 1, 1], ">=": [0, 0, 1, 1, 1, 1], ">": [0, 0, 0, 0, 1, 1]}[cmp]
    assert oracle_mod.view_update(col, 1, 7, pred=p, cmp=cmp, thr=3).tolist() == \
        [7 * t for t in take]
    pf = p.astype(np.float32)
    colf = np.zeros(6, dtype=np.float32)
    assert oracle_mod.view_update(colf, 1, 0.5, pred=pf, cmp=cmp, thr=3.0).tolist() == \
        [0.5 * t for t in take]


def test_filtered_float_predicate_with_nan(oracle_mod):
    p = np.array([np.nan, 1.0, np.nan], dtype=np.float32)
    col = np.zeros(3, dtype=np.int32)
    for cmp in CMPS:
        got = oracle_mod.view_update(col, 1, 1, pred=p, cmp=cmp, thr=1.0)
        nan_rows = [got[0], got[2]]
        assert nan_rows == ([1, 1] if cmp == "!=" else [0, 0]), cmp


@pytest.mark.parametrize("seed", range(4))
def test_scatter_add_int32_matches_numpy_add_at(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n, m = 300, 5000
    col = rng.integers(-1000, 1000, n).astype(np.int32)
    ids = rng.integers(0, n + 20, m).astype(np.uint32)          # some out of range
    vals = rng.integers(-2**31, 2**31, m, dtype=np.int64).astype(np.int32)
    keep = ids < n
    want = col.copy()
    with np.errstate(over="ignore"):
        np.add.at(want, ids[keep], vals[keep])
    assert np.array_equal(oracle_mod.scatter_add(col, ids, vals), want)
    # a scalar per entry; the hammer (every entry on one id)
    want = col.copy()
    np.add.at(want, ids[keep], np.int32(3))
    assert np.array_equal(oracle_mod.scatter_add(col, ids, scalar=3), want)
    hammer = oracle_mod.scatter_add(col, np.full(m, 7, np.uint32), scalar=-2)
    assert hammer[7] == col[7] - 2 * m and np.array_equal(np.delete(hammer, 7), np.delete(col, 7))


@pytest.mark.parametrize("seed", range(4))
def test_scatter_add_float32_in_list_order(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n, m = 50, 4000
    col = rng.standard_normal(n).astype(np.float32)
    ids = rng.integers(0, n, m).astype(np.uint32)
    vals = (rng.standard_normal(m) * 10.0 ** rng.integers(-3, 6, m)).astype(np.float32)
    want = col.copy()
    np.add.at(want, ids, vals)               # float32, unbuffered, in list order
    assert np.array_equal(oracle_mod.scatter_add(col, ids, vals), want)
    # order decides (float32 spacing is 8 at 1e8): ((0 + 1e8) + 4) + 4 = 1e8
    # (each half-way sum rounds to the even 1e8), while (4 + 4) + 1e8 = 1e8 + 8
    got = oracle_mod.scatter_add(np.zeros(1, np.float32), [0, 0, 0],
                                 np.array([1e8, 4, 4], np.float32))
    assert got[0] == np.float32(1e8)
    got = oracle_mod.scatter_add(np.zeros(1, np.float32), [0, 0, 0],
                                 np.array([4, 4, 1e8], np.float32))
    assert got[0] == np.float32(100000008) and np.float32(100000008) != np.float32(1e8)


@pytest.mark.parametrize("model", [0, 1, 2])
def test_resumed_run_equals_the_single_run(oracle_mod, model):
    n, L, T, t = 3001, 41, 30, 11
    kw = dict(seed=3, stream=8, beta=(1, 4), gamma=(1, 30))
    whole = oracle_mod.OracleRun(model, n, L, **kw).step(T)
    first = oracle_mod.OracleRun(model, n, L, **kw).step(t)
    rest = oracle_mod.OracleRun.resume(model, first.columns(), t, L, **kw).step(T - t)
    assert rest.t == T
    for a, b in zip(whole.columns(), rest.columns()):
        assert np.array_equal(a, b)
    assert whole.digest() == rest.digest()
