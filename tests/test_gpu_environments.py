"""GPU parity of the environment primitives (Sec. 4.1) against the oracle:
n-D grid binning, Moore / von Neumann neighbour sums (torus and bounded,
sides down to 1), per-agent gathers, network neighbour counts over ER, WS
and BA graphs, and the SIR transition alone; then two SIR variants composed
from them: the grid SIR rebuilt step by step (equal to the model's own
step), a von Neumann grid SIR and a network SIR (equal to the oracle's
composition of the same primitives)."""
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


GRIDS = [((7,), 40), ((1,), 5), ((2,), 9), ((5, 4), 60), ((2, 3), 300), ((1, 6), 20),
         ((3, 3, 3), 800), ((4, 2, 5), 700), ((3, 2, 2, 3), 600), ((2, 2, 2, 2), 400),
         ((1000, 1000), 1_000_000), ((64, 64, 64), 500_000), ((20, 20, 20, 20), 300_001)]


@pytest.mark.parametrize("dims,n", GRIDS)
@pytest.mark.parametrize("vn", [False, True])
@pytest.mark.parametrize("torus", [True, False])
def test_grid_primitives(A, O, dims, n, vn, torus):
    say(f"case grid dims={dims} n={n} vn={vn} torus={torus}")
    rng = np.random.default_rng(sum(dims) + n)
    pos = [rng.integers(0, d, n).astype(np.int32) for d in dims]
    pos[-1][:2] = [-1, dims[-1]]
    state = rng.integers(0, 3, n).astype(np.uint8)
    dpos = [dev(p) for p in pos]
    C = A.grid_count(dims, dpos, dev(state), 1)
    Cw = O.grid_count(dims, pos, state, 1)
    assert np.array_equal(host(C).view(np.uint32), Cw)
    K = A.grid_neighbour_sum(dims, C, A.VON_NEUMANN if vn else A.MOORE, torus)
    Kw = O.grid_neighbour_sum(dims, Cw, von_neumann=vn, torus=torus)
    assert np.array_equal(host(K).view(np.uint32), Kw)
    k = A.grid_gather(dims, dpos, K)
    assert np.array_equal(host(k).view(np.uint32), O.grid_gather(dims, pos, Kw))
    Call = A.grid_count(dims, dpos)
    assert np.array_equal(host(Call).view(np.uint32), O.grid_count(dims, pos, None))


@pytest.mark.parametrize("kind,n", [("er", 3000), ("ws", 20000), ("ba", 20000), ("ba", 100)])
def test_graph_counts(A, O, kind, n):
    from paper_2601_16292_amd import workloads as W
    say(f"case graph {kind} n={n}")
    row, col = W.graph_csr(kind, n, seed=3)
    s = np.random.default_rng(1).integers(0, 3, n).astype(np.uint8)
    got = A.graph_neighbour_count(dev(row.view(np.int32)), dev(col.view(np.int32)), dev(s), 1)
    assert np.array_equal(host(got).view(np.uint32), O.graph_count(row, col, s, 1))


def test_graph_counts_large_multigraph(A, O):
    from paper_2601_16292_amd import workloads as W
    say("case graph random multigraph n=2^20")
    n = 1 << 20
    row, col = W.random_graph_csr(n, 10, seed=4)
    col[::1001] = n + 5                                     # entries naming no node
    s = np.random.default_rng(2).integers(0, 3, n).astype(np.uint8)
    got = A.graph_neighbour_count(dev(row.view(np.int32)), dev(col.view(np.int32)), dev(s), 2)
    assert np.array_equal(host(got).view(np.uint32), O.graph_count(row, col, s, 2))


@pytest.mark.parametrize("n", [1, 3, 5, 4097, 1_000_003])
def test_sir_transition(A, O, n):
    say(f"case SIR transition n={n}")
    rng = np.random.default_rng(n)
    s = rng.integers(0, 3, n).astype(np.uint8)
    k = rng.integers(0, 12, n).astype(np.uint32)
    ds = dev(s)
    A.sir_transition(ds, dev(k.view(np.int32)), 7, 8, 9, beta=(1, 5), gamma=(1, 20))
    assert np.array_equal(host(ds), O.sir_transition(s, k, 7, 8, 9, beta=(1, 5), gamma=(1, 20)))


def _walk_move(A, x, y, L, seed, stream, t):
    """The SIR move of step t: the random walk's step t from (x, y)."""
    p = A.Population(A.RANDOM_WALK, len(x), L=L, seed=seed, stream_id=stream,
                     resume=([x, y], t))
    p.step(1)
    nx, ny = p.read()
    p.release()
    return nx, ny


@pytest.mark.parametrize("n,L,steps", [(40000, 200, 15), (3000, 2, 6)])
def test_grid_sir_rebuilt_from_primitives_equals_the_model(A, O, n, L, steps):
    say(f"case SIR from primitives n={n} L={L}")
    beta, gamma = (1, 4), (1, 30)
    ref = O.OracleRun(O.SIR, n, L, seed=3, stream=4, beta=beta, gamma=gamma)
    x, y, s = (c.copy() for c in ref.columns())
    ds = dev(s)
    for t in range(steps):
        x, y = _walk_move(A, x, y, L, 3, 4, t)
        dx, dy = dev(x), dev(y)
        C = A.grid_count((L, L), [dx, dy], ds, 1)
        k = A.grid_gather((L, L), [dx, dy], A.grid_neighbour_sum((L, L), C))
        A.sir_transition(ds, k, 3, 4, t, beta=beta, gamma=gamma)
        ref.step(1)
    assert np.array_equal(host(ds), ref.s)


@pytest.mark.parametrize("variant", ["von_neumann_bounded", "network_ba"])
def test_sir_variants_match_the_oracle_composition(A, O, variant):
    from paper_2601_16292_amd import workloads as W
    say(f"case SIR variant {variant}")
    beta, gamma, seed, stream, steps = (1, 3), (1, 25), 5, 6, 12
    n, L = 30000, 150
    rng = np.random.default_rng(9)
    s = np.zeros(n, np.uint8)
    s[:30] = 1
    if variant == "network_ba":
        row, col = W.graph_csr("ba", n, seed=2)
        drow, dcol, ds = dev(row.view(np.int32)), dev(col.view(np.int32)), dev(s)
        sw = s.copy()
        for t in range(steps):
            k = A.graph_neighbour_count(drow, dcol, ds, 1)
            A.sir_transition(ds, k, seed, stream, t, beta=beta, gamma=gamma)
            kw = O.graph_count(row, col, sw, 1)
            sw = O.sir_transition(sw, kw, seed, stream, t, beta=beta, gamma=gamma)
        assert np.array_equal(host(ds), sw)
        assert (sw != 0).sum() > 30                       # the epidemic spread
        return
    x = rng.integers(0, L, n).astype(np.int32)
    y = rng.integers(0, L, n).astype(np.int32)
    ds, sw = dev(s), s.copy()
    for t in range(steps):
        x, y = _walk_move(A, x, y, L, seed, stream, t)
        dx, dy = dev(x), dev(y)
        C = A.grid_count((L, L), [dx, dy], ds, 1)
        K = A.grid_neighbour_sum((L, L), C, A.VON_NEUMANN, torus=False)
        A.sir_transition(ds, A.grid_gather((L, L), [dx, dy], K), seed, stream, t, beta=beta,
                         gamma=gamma)
        Cw = O.grid_count((L, L), [x, y], sw, 1)
        kw = O.grid_gather((L, L), [x, y], O.grid_neighbour_sum((L, L), Cw, von_neumann=True,
                                                                torus=False))
        sw = O.sir_transition(sw, kw, seed, stream, t, beta=beta, gamma=gamma)
    assert np.array_equal(host(ds), sw)
