"""GPU parity of the buffered write log (the pending-writes flush of
Sec. 3.2.1) and of asynchronous (sequential) update semantics (Sec. 3.4)
against the oracle, bit for bit."""
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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,m", [(1, 1), (1, 5), (10, 3), (300, 5000), (4097, 2049),
                                 (100_003, 250_007), (1_000_000, 3_000_000)])
@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_write_log_last_write_wins(A, O, n, m, dtype):
    say(f"case write log n={n} m={m} dtype={dtype.__name__}")
    rng = np.random.default_rng(n * 7 + m)
    col = rng.integers(-1000, 1000, n).astype(dtype)
    ids = rng.integers(0, n + max(1, n // 40), m).astype(np.uint32)
    vals = rng.integers(-10**6, 10**6, m).astype(dtype)
    if dtype == np.float32:
        vals[::5] = -0.0
    t = dev(col)
    A.write_log(t, dev(ids.view(np.int32)), dev(vals))
    got, want = host(t), O.write_log(col, ids, vals)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_write_log_hammered_id(A, O):
    say("case write log hammer")
    m = 200_000
    ids = np.full(m, 17, np.uint32)
    vals = np.arange(m, dtype=np.int32)
    t = dev(np.zeros(50, np.int32))
    A.write_log(t, dev(ids.view(np.int32)), dev(vals))
    got = host(t)
    assert got[17] == m - 1 and np.array_equal(got, O.write_log(np.zeros(50, np.int32), ids, vals))


@pytest.mark.parametrize("n,w0,steps,chunks", [(1, 3, 5, [5]), (2, 1, 9, [4, 5]),
                                               (1000, 1, 100, [100]), (1000, 1, 30, [7, 23]),
                                               (20011, 2, 12, [12]), (100_003, 1, 8, [3, 5])])
def test_async_wealth_matches_oracle(A, O, n, w0, steps, chunks):
    say(f"case async wealth n={n} w0={w0} steps={steps} chunks={chunks}")
    pop = A.Population(A.WEALTH, n, seed=3, stream_id=n % 11, wealth_init=w0)
    for c in chunks:
        pop.step_async(c)
    (w,), inv = pop.read(), pop.invariants()
    pop.release()
    want = O.run_wealth_async(np.full(n, w0, np.int32), 3, n % 11, 0, steps)
    assert np.array_equal(w, want)
    assert inv["step"] == steps and inv["wealth_sum"] == n * w0 and inv["wealth_min"] >= 0
    assert inv["digest"] == O.digest([want])


def test_async_and_sync_steps_alternate(A, O):
    say("case async and sync alternate")
    n = 30001
    pop = A.Population(A.WEALTH, n, seed=9, stream_id=4, wealth_init=1)
    pop.step(3)
    pop.step_async(4)
    pop.step(2)
    pop.step_async(1)
    (w,) = pop.read()
    pop.release()
    ref = O.OracleRun(O.WEALTH, n, seed=9, stream=4, wealth_init=1).step(3)
    want = O.run_wealth_async(ref.w, 9, 4, 3, 4)
    ref2 = O.OracleRun.resume(O.WEALTH, [want], 7, seed=9, stream=4).step(2)
    want = O.run_wealth_async(ref2.w, 9, 4, 9, 1)
    assert np.array_equal(w, want)


def test_async_random_walk_is_the_synchronous_step(A, O):
    say("case async random walk")
    pop = A.Population(A.RANDOM_WALK, 4099, L=37, seed=1, stream_id=2)
    pop.step_async(20)
    x, y = pop.read()
    pop.release()
    ref = O.OracleRun(O.RANDOM_WALK, 4099, 37, seed=1, stream=2).step(20)
    assert np.array_equal(x, ref.x) and np.array_equal(y, ref.y)


def test_async_sir_is_unsupported(A):
    pop = A.Population(A.SIR, 1000)
    with pytest.raises(A.AmberError) as e:
        pop.step_async(1)
    assert e.value.status == A.E_UNSUPPORTED
    pop.release()
