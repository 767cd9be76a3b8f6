"""GPU parity of the view primitives (Sec. 3.3 views, Sec. 3.1.1 listings)
and of resuming a run from host columns, against the oracle, bit for bit:
full and filtered updates on int32 / float32 columns (every comparison,
predicates of either type, aligned and unaligned columns, sizes across many
workgroups with ragged tails), int32 and float32 scatter-adds (duplicates,
ids outside the column, one id hammered, float32 values whose sum depends on
the order), a wealth step composed from the views, and split runs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2601_16292_amd import amber
    amber.lib()
    return amber


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def say(*a):
    print(*a, flush=True)


def dev(a, offset=0):
    """Device copy of a numpy array; offset > 0 gives a view that starts
    `offset` elements into its allocation (4-byte but not 16-byte aligned)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if offset:
        pad = torch.zeros(len(a) + offset, dtype=t.dtype)
        pad[offset:] = t
        return pad.cuda()[offset:]
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


SIZES = [1, 3, 4, 5, 1023, 4097, 1_000_003]


def _col(rng, dtype, n):
    if dtype == np.int32:
        return rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)
    return (rng.standard_normal(n) * 10.0 ** rng.integers(-3, 4, n)).astype(np.float32)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype", [np.int32, np.float32])
@pytest.mark.parametrize("offset", [0, 1])
def test_full_view_update(A, O, n, dtype, offset):
    say(f"case view full n={n} dtype={dtype.__name__} offset={offset}")
    rng = np.random.default_rng(n)
    col = _col(rng, dtype, n)
    a, b = (int(rng.integers(-1000, 1000)), int(rng.integers(-2**31, 2**31))) \
        if dtype == np.int32 else (np.float32(1.0001), np.float32(-2.5))
    t = dev(col, offset)
    A.view_update(t, a, b)
    assert np.array_equal(host(t), O.view_update(col, a, b))


@pytest.mark.parametrize("cmp", ["<", "<=", "==", "!=", ">=", ">"])
@pytest.mark.parametrize("dtype,pdtype", [(np.int32, np.int32), (np.int32, np.float32),
                                          (np.float32, np.int32), (np.float32, np.float32)])
def test_filtered_view_update(A, O, cmp, dtype, pdtype):
    for n, offset in ((4097, 0), (70001, 1)):
        say(f"case view filtered cmp={cmp} {dtype.__name__}/{pdtype.__name__} n={n}")
        rng = np.random.default_rng(len(cmp) + n)
        col = _col(rng, dtype, n)
        pred = rng.integers(-5, 6, n).astype(pdtype)
        if pdtype == np.float32:
            pred[::7] = np.nan
        a, b = (3, -7) if dtype == np.int32 else (np.float32(0.5), np.float32(1.25))
        t, p = dev(col, offset), dev(pred, offset)
        A.view_update(t, a, b, pred=p, cmp=cmp, thr=2)
        assert np.array_equal(host(t), O.view_update(col, a, b, pred=pred, cmp=cmp, thr=2))


def test_filtered_update_on_its_own_column(A, O):
    say("case view filtered on itself (donors give one)")
    w = np.random.default_rng(5).integers(-2, 4, 100_001).astype(np.int32)
    t = dev(w)
    A.view_update(t, 1, -1, pred=t, cmp=">", thr=0)
    assert np.array_equal(host(t), O.view_update(w, 1, -1, pred=w, cmp=">", thr=0))


@pytest.mark.parametrize("n,m", [(1, 1), (7, 1000), (300, 5000), (100_003, 250_007),
                                 (1_000_000, 3_000_000)])
def test_scatter_add_int32(A, O, n, m):
    say(f"case scatter int32 n={n} m={m}")
    rng = np.random.default_rng(m)
    col = rng.integers(-1000, 1000, n).astype(np.int32)
    ids = rng.integers(0, n + max(1, n // 50), m).astype(np.uint32)
    vals = rng.integers(-2**31, 2**31, m, dtype=np.int64).astype(np.int32)
    t = dev(col)
    A.scatter_add(t, dev(ids.view(np.int32)), dev(vals))
    assert np.array_equal(host(t), O.scatter_add(col, ids, vals))
    t = dev(col)
    A.scatter_add(t, dev(ids.view(np.int32)), scalar=1)
    assert np.array_equal(host(t), O.scatter_add(col, ids, scalar=1))


@pytest.mark.parametrize("n,m", [(1, 1), (1, 3), (7, 1000), (300, 5000), (4099, 20_000),
                                 (100_003, 250_007), (1_000_000, 3_000_000), (70_000, 2049)])
def test_scatter_add_float32_in_list_order(A, O, n, m):
    say(f"case scatter float32 n={n} m={m}")
    rng = np.random.default_rng(n + m)
    col = _col(rng, np.float32, n)
    ids = rng.integers(0, n + max(1, n // 50), m).astype(np.uint32)
    vals = _col(rng, np.float32, m)
    t = dev(col)
    A.scatter_add(t, dev(ids.view(np.int32)), dev(vals))
    assert np.array_equal(host(t), O.scatter_add(col, ids, vals))
    t = dev(col)
    A.scatter_add(t, dev(ids.view(np.int32)), scalar=np.float32(0.1))
    assert np.array_equal(host(t), O.scatter_add(col, ids, scalar=np.float32(0.1)))


def test_scatter_add_float32_order_and_hammer(A, O):
    say("case scatter float32 order and hammer")
    t = dev(np.zeros(1, np.float32))
    A.scatter_add(t, dev(np.zeros(3, np.int32)), dev(np.array([1e8, 4, 4], np.float32)))
    assert host(t)[0] == np.float32(1e8)
    t = dev(np.zeros(1, np.float32))
    A.scatter_add(t, dev(np.zeros(3, np.int32)), dev(np.array([4, 4, 1e8], np.float32)))
    assert host(t)[0] == np.float32(100000008)
    rng = np.random.default_rng(2)
    n, m = 1000, 100_000
    col = _col(rng, np.float32, n)
    ids = np.full(m, 321, np.uint32)
    ids[::3] = rng.integers(0, n, len(ids[::3]))
    vals = _col(rng, np.float32, m)
    t = dev(col)
    A.scatter_add(t, dev(ids.view(np.int32)), dev(vals))
    assert np.array_equal(host(t), O.scatter_add(col, ids, vals))


@pytest.mark.parametrize("n,steps", [(1000, 3), (100_003, 4)])
def test_wealth_step_composed_from_the_views(A, O, n, steps):
    """The wealth rule as the paper's listings write it: donors (wealth > 0)
    give one unit through a filtered view, and recipients (the oracle's
    RECIPIENT draws of the donors) receive through the scatter view.  Equal
    to the oracle's wealth run, step after step."""
    say(f"case wealth from views n={n} steps={steps}")
    ref = O.OracleRun(O.WEALTH, n, seed=4, stream=2, wealth_init=2)
    t = dev(np.full(n, 2, np.int32))
    for s in range(steps):
        w = host(t)
        donors = np.flatnonzero(w > 0)
        rec = np.array([O.recipient(n, 4, 2, s, int(a)) for a in donors], dtype=np.uint32)
        A.view_update(t, 1, -1, pred=t, cmp=">", thr=0)
        A.scatter_add(t, dev(rec.view(np.int32)), scalar=1)
        ref.step(1)
        assert np.array_equal(host(t), ref.w), s


@pytest.mark.parametrize("model,n,L,T,t", [(0, 20011, 0, 9, 4), (0, 1000, 0, 100, 37),
                                           (1, 70001, 265, 40, 13), (2, 40000, 200, 90, 31),
                                           (2, 5003, 71, 25, 24)])
def test_resumed_run_equals_the_oracle(A, O, model, n, L, T, t):
    say(f"case resume model={model} n={n} L={L} T={T} t={t}")
    kw = dict(seed=6, stream_id=3, beta=(1, 4), gamma=(1, 30))
    first = A.Population(model, n, L=L, **kw)
    first.step(t)
    cols = first.read()
    first.release()
    pop = A.Population(model, n, L=L, resume=(cols, t), **kw)
    assert pop.info().step == t
    pop.step(T - t)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    ref = O.OracleRun(model, n, L, seed=6, stream=3, beta=(1, 4), gamma=(1, 30)).step(T)
    for g, r in zip(got, ref.columns()):
        assert np.array_equal(g, r)
    assert inv["step"] == T and inv["digest"] == ref.digest()
    # resumed from the oracle's own state at t as well
    mid = O.OracleRun(model, n, L, seed=6, stream=3, beta=(1, 4), gamma=(1, 30)).step(t)
    pop = A.Population(model, n, L=L, resume=(mid.columns(), t), **kw)
    pop.step(T - t)
    assert pop.invariants()["digest"] == ref.digest()
    pop.release()
