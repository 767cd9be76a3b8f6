"""GPU parity of the paper's continuous-space models (Sec. 5.1.2) against the
oracle's all-pairs definition, bit for bit: the clamped random walk and the
SIR with contacts within radius r (cell list on the GPU), at the paper's
sizes (N = 500, 1000, 5000, 50 steps, 100 x 100, r = 5, p = 0.1, recovery
after 14 days, five initially infected) and others (denser and sparser
worlds, cell-aligned sides, chunked calls)."""
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


@pytest.mark.parametrize("n,W,steps,chunks", [(500, 100.0, 50, [50]), (5000, 100.0, 50, [20, 30]),
                                              (1, 3.0, 7, [7]), (200_003, 1000.0, 100, [100]),
                                              (4097, 0.0, 5, [5])])
def test_continuous_walk(A, O, n, W, steps, chunks):
    say(f"case continuous walk n={n} W={W} steps={steps}")
    g = A.ContRun(n, W=W, seed=1, stream_id=2)
    for c in chunks:
        g.step(c)
    x, y = g.read()
    ref = O.ContRun(O.RANDOM_WALK, n, W=W, seed=1, stream=2).step(steps)
    assert np.array_equal(x, ref.x) and np.array_equal(y, ref.y)


SIR_CASES = [
    (500, 100.0, 5.0, (1, 10), 14, 5, 50, [50]),        # the paper's sizes
    (1000, 100.0, 5.0, (1, 10), 14, 5, 50, [50]),
    (5000, 100.0, 5.0, (1, 10), 14, 5, 50, [25, 25]),
    (3000, 30.0, 2.0, (1, 4), 6, 40, 40, [40]),          # denser, faster epidemic
    (2000, 40.0, 4.0, (1, 3), 9, 10, 30, [13, 17]),      # W / r an integer: agents on the last cell
    (800, 5.0, 7.5, (1, 20), 3, 2, 12, [12]),            # radius wider than the world
    (6000, 1000.0, 5.0, (1, 2), 14, 300, 20, [20]),      # sparse
]


@pytest.mark.parametrize("n,W,r,p,recover,i0,steps,chunks", SIR_CASES)
def test_continuous_sir(A, O, n, W, r, p, recover, i0, steps, chunks):
    say(f"case continuous SIR n={n} W={W} r={r} p={p} recover={recover} i0={i0} steps={steps}")
    g = A.ContRun(n, W=W, r=r, seed=4, stream_id=9, sir=True, p=p, recover=recover,
                  initial_infected=i0)
    for c in chunks:
        g.step(c)
    x, y, s, d = g.read()
    ref = O.ContRun(O.SIR, n, W=W, r=r, seed=4, stream=9, p=p, recover=recover,
                    initial_infected=i0).step(steps)
    assert np.array_equal(x, ref.x) and np.array_equal(y, ref.y)
    assert np.array_equal(s, ref.s), (np.flatnonzero(s != ref.s)[:8])
    assert np.array_equal(d, ref.days)
    assert (s != 0).sum() > i0 or p[0] == 0               # the epidemic did spread
