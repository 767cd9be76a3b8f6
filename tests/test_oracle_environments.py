"""Pins of the oracle's spatial environments (Sec. 4.1): n-D grids with
Moore or von Neumann neighbourhoods, torus-wrapped or bounded, and network
neighbour counts over adjacency lists; and of the SIR transition on its own.

  * grid neighbour sums against a brute force over agent pairs that tests a
    per-axis distance (Chebyshev for Moore, Manhattan for von Neumann, the
    short way round on a torus) instead of enumerating cells;
  * the 2-D Moore torus case against the SIR model's own neighbour count;
  * network counts against scipy's sparse matrix-vector product and, on
    small graphs, NetworkX's neighbour lists;
  * the primitives composed (move, bin, neighbour sum, gather, transition)
    against the SIR model's step.
"""
import numpy as np
import pytest


def _brute_k(dims, pos, state, von_neumann, torus):
    n = len(pos[0])
    P = np.stack(pos, axis=1).astype(np.int64)
    dims = np.array(dims, dtype=np.int64)
    inside = np.all((P >= 0) & (P < dims), axis=1)
    k = np.zeros(n, dtype=np.int64)
    inf = np.flatnonzero((state == 1) & inside)
    for a in range(n):
        if not inside[a]:
            continue
        d = np.abs(P[inf] - P[a])
        if torus:
            d = np.minimum(d, dims - d)
        near = d.sum(axis=1) <= 1 if von_neumann else d.max(axis=1) <= 1
        k[a] = int(near.sum())
    return k


CASES = [((7,), 40), ((1,), 5), ((2,), 9), ((5, 4), 60), ((2, 3), 30), ((1, 6), 20),
         ((3, 3, 3), 80), ((4, 2, 5), 70), ((3, 2, 2, 3), 60), ((2, 2, 2, 2), 40)]


@pytest.mark.parametrize("dims,n", CASES)
@pytest.mark.parametrize("vn", [False, True])
@pytest.mark.parametrize("torus", [True, False])
def test_grid_neighbour_counts_match_pairwise_distances(oracle_mod, dims, n, vn, torus):
    rng = np.random.default_rng(sum(dims) * 31 + n)
    pos = [rng.integers(0, d, n).astype(np.int32) for d in dims]
    pos[0][:2] = [-1, dims[0]]                  # two agents off the lattice
    state = rng.integers(0, 3, n).astype(np.uint8)
    C = oracle_mod.grid_count(dims, pos, state, 1)
    K = oracle_mod.grid_neighbour_sum(dims, C, von_neumann=vn, torus=torus)
    k = oracle_mod.grid_gather(dims, pos, K)
    assert np.array_equal(k.astype(np.int64), _brute_k(dims, pos, state, vn, torus))


def test_grid_count_all_agents_and_bounds(oracle_mod):
    pos = [np.array([0, 1, 1, 5, -1], np.int32), np.array([0, 0, 0, 1, 0], np.int32)]
    C = oracle_mod.grid_count((5, 2), pos, None)
    assert C.tolist() == [1, 2, 0, 0, 0, 0, 0, 0, 0, 0]


@pytest.mark.parametrize("L", [1, 2, 3, 7])
def test_moore_torus_2d_is_the_sir_count(oracle_mod, L):
    rng = np.random.default_rng(L)
    n = 200
    x = rng.integers(0, L, n).astype(np.int32)
    y = rng.integers(0, L, n).astype(np.int32)
    s = rng.integers(0, 3, n).astype(np.uint8)
    C = oracle_mod.grid_count((L, L), [x, y], s, 1)
    k = oracle_mod.grid_gather((L, L), [x, y], oracle_mod.grid_neighbour_sum((L, L), C))
    for a in range(n):
        assert k[a] == oracle_mod.neighbour_infected(L, C, int(x[a]), int(y[a]))


@pytest.mark.parametrize("kind", ["er", "ws", "ba"])
def test_graph_counts_match_sparse_product_and_networkx(oracle_mod, kind):
    import networkx as nx
    import scipy.sparse as sp
    from paper_2601_16292_amd import workloads as W
    n = 3000
    row, col = W.graph_csr(kind, n, seed=5)
    s = np.random.default_rng(2).integers(0, 3, n).astype(np.uint8)
    got = oracle_mod.graph_count(row, col, s, 1)
    A = sp.csr_matrix((np.ones(len(col)), col.astype(np.int64), row.astype(np.int64)), shape=(n, n))
    assert np.array_equal(got, (A @ (s == 1).astype(np.float64)).astype(np.uint32))
    g = {"er": lambda: nx.gnm_random_graph(n, n * 3, seed=5),
         "ws": lambda: nx.watts_strogatz_graph(n, 6, 0.1, seed=5),
         "ba": lambda: nx.barabasi_albert_graph(n, 3, seed=5)}[kind]()
    for i in range(0, n, 97):
        assert got[i] == sum(1 for j in g.neighbors(i) if s[j] == 1)


def test_graph_count_repeats_and_out_of_range(oracle_mod):
    row = np.array([0, 3, 3, 5], np.uint32)
    col = np.array([1, 1, 2, 0, 9], np.uint32)          # node 0 lists 1 twice; 9 is no node
    s = np.array([1, 1, 0], np.uint8)
    assert oracle_mod.graph_count(row, col, s, 1).tolist() == [2, 0, 1]


def test_sir_transition_special_cases(oracle_mod):
    n = 10000
    s = np.random.default_rng(0).integers(0, 3, n).astype(np.uint8)
    k = np.random.default_rng(1).integers(0, 5, n).astype(np.uint32)
    got = oracle_mod.sir_transition(s, k, 1, 2, 3, beta=(0, 1), gamma=(0, 1))
    assert np.array_equal(got, s)                           # no infection, no recovery
    got = oracle_mod.sir_transition(s, np.zeros(n, np.uint32), 1, 2, 3)
    assert np.array_equal(got[s == 0], s[s == 0])           # k = 0 never infects
    assert (got[s == 2] == 2).all()                         # R is absorbing
    assert set(np.unique(got[s == 1]).tolist()) <= {1, 2}


@pytest.mark.parametrize("n,L,steps", [(3000, 41, 12), (500, 2, 6), (2000, 97, 20)])
def test_primitives_compose_into_the_sir_step(oracle_mod, n, L, steps):
    ref = oracle_mod.OracleRun(oracle_mod.SIR, n, L, seed=3, stream=4, beta=(1, 4),
                               gamma=(1, 30))
    x, y, s = (c.copy() for c in ref.columns())
    for t in range(steps):
        mv = oracle_mod.OracleRun.resume(oracle_mod.RANDOM_WALK, [x, y], t, L, seed=3,
                                         stream=4).step(1)
        x, y = mv.x, mv.y
        C = oracle_mod.grid_count((L, L), [x, y], s, 1)
        k = oracle_mod.grid_gather((L, L), [x, y], oracle_mod.grid_neighbour_sum((L, L), C))
        s = oracle_mod.sir_transition(s, k, 3, 4, t, beta=(1, 4), gamma=(1, 30))
        ref.step(1)
        assert np.array_equal(x, ref.x) and np.array_equal(y, ref.y)
        assert np.array_equal(s, ref.s), t
