"""Seeded synthetic workloads (inputs only; none of the model arithmetic).

Shared by the GPU path's tests and benchmark and by the oracle's tests: the
paper has no datasets, so every input is generated here from fixed seeds with
the shapes the workloads call for.  Run sizes, step counts, parameters and
arrival times are produced with numpy's PCG64 generator; grid sides and
initial infected counts are left to each side's own defaults.
"""
import numpy as np

# -------------------------------------------------------------- single runs

# Boltzmann wealth transfer: N = 1000, wealth 1 each, 100 steps, key (0, 0).
WEALTH_1K = dict(model=0, n=1000, steps=100, wealth_init=1, seed=0, stream=0)
# Torus random walk: N = 1e6 on 1000 x 1000, 1000 steps.
WALK_1M = dict(model=1, n=1_000_000, L=1000, steps=1000, seed=0, stream=0)
# Grid SIR: N = 1e6 on 1000 x 1000, beta 1/20, gamma 1/100, 0.1% infected, 500 steps.
SIR_1M = dict(model=2, n=1_000_000, L=1000, steps=500, beta=(1, 20), gamma=(1, 100),
              seed=0, stream=0)

# Out-of-cache shapes for roofline measurements (columns far above the
# 256 MB last-level cache).
WALK_BIG = dict(model=1, n=1 << 27, L=1000, seed=0, stream=0)
SIR_BIG = dict(model=2, n=1 << 27, L=0, beta=(1, 20), gamma=(1, 100), seed=0, stream=0)
WEALTH_BIG = dict(model=0, n=1 << 27, wealth_init=1, seed=0, stream=0)

# -------------------------------------------------------------- SIR sweep

SWEEP_BETAS = [(15 + 19 * j, 1500) for j in range(16)]   # 16 linear values 0.01 .. 0.2


def sir_sweep(n_runs=256, steps=300, seed=0x5EED_0004, n_lo=1e3, n_hi=1e6):
    """256 SIR replicates: N log-uniform in [n_lo, n_hi], beta_j for
    j = r // (n_runs/16), gamma 1/100, key (0, r)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(n_runs)
    ns = np.rint(10 ** (np.log10(n_lo) + (np.log10(n_hi) - np.log10(n_lo)) * u)).astype(np.int64)
    per_beta = max(1, n_runs // len(SWEEP_BETAS))
    runs = []
    for r in range(n_runs):
        runs.append(dict(model=2, n=int(ns[r]), L=0, steps=steps,
                         beta=SWEEP_BETAS[min(r // per_beta, len(SWEEP_BETAS) - 1)],
                         gamma=(1, 100), seed=0, stream=r))
    return runs


# -------------------------------------------------------------- served stream

def served_stream(n_requests=10_000, rate_per_s=50.0, seed=0x5EED_0005, n_lo=1e4, n_hi=1e7,
                  steps_lo=100, steps_hi=1000):
    """Poisson arrivals (exponential gaps, mean 1/rate) of wealth, random-walk
    and SIR runs (uniform mix), N log-uniform in [n_lo, n_hi], steps uniform
    in [steps_lo, steps_hi], key (0, request id)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    arrivals = np.cumsum(gaps)
    models = rng.integers(0, 3, n_requests)
    u = rng.random(n_requests)
    ns = np.rint(10 ** (np.log10(n_lo) + (np.log10(n_hi) - np.log10(n_lo)) * u)).astype(np.int64)
    steps = rng.integers(steps_lo, steps_hi + 1, n_requests)
    reqs = []
    for i in range(n_requests):
        m = int(models[i])
        req = dict(id=i, arrival=float(arrivals[i]), model=m, n=int(ns[i]), steps=int(steps[i]),
                   seed=0, stream=i, L=0)
        if m == 0:
            req["wealth_init"] = 1
        if m == 2:
            req["beta"], req["gamma"] = (1, 20), (1, 100)
        reqs.append(req)
    return reqs


# -------------------------------------------------------------- networks

def graph_csr(kind, n, seed=0, degree=6, rewire=0.1):
    """Undirected network of n nodes as CSR arrays (row offsets uint32[n+1],
    neighbour ids uint32[2 |E|], each edge listed from both ends), for the
    network environment's three generators: "er" (Erdos-Renyi G(n, M) with
    M = n * degree / 2 distinct edges), "ws" (Watts-Strogatz: ring lattice of
    `degree` neighbours, each edge rewired with probability `rewire`), "ba"
    (Barabasi-Albert, degree / 2 edges per new node).  Generated with
    NetworkX (the paper's network library) from a fixed seed."""
    import networkx as nx
    if kind == "er":
        g = nx.gnm_random_graph(n, n * degree // 2, seed=seed)
    elif kind == "ws":
        g = nx.watts_strogatz_graph(n, degree, rewire, seed=seed)
    elif kind == "ba":
        g = nx.barabasi_albert_graph(n, max(1, degree // 2), seed=seed)
    else:
        raise ValueError(kind)
    e = np.array(g.edges(), dtype=np.int64).reshape(-1, 2)
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row = np.zeros(n + 1, dtype=np.uint32)
    np.add.at(row, src + 1, 1)
    return np.cumsum(row, dtype=np.uint32), dst.astype(np.uint32)


def random_graph_csr(n, degree, seed=0):
    """A large random multigraph for throughput runs: n * degree / 2 edges
    with both ends uniform over the nodes (self loops and repeats kept, as
    adjacency entries), as CSR arrays; numpy's PCG64 from a fixed seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = n * degree // 2
    a = rng.integers(0, n, m, dtype=np.int64)
    b = rng.integers(0, n, m, dtype=np.int64)
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order = np.argsort(src, kind="stable")
    src, dst = src[order], dst[order]
    row = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row, src + 1, 1)
    return np.cumsum(row).astype(np.uint32), dst.astype(np.uint32)
