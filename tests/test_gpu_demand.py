"""GPU parity of the gather mode's demand-driven binning: once susceptible
agents are few next to many infected ones (32 S <= I and 10 I >= N, three
steps back), infected
agents are binned only on cells a susceptible agent may read.  Every count
that is read must still be exact, so results equal the oracle bit for bit.
Each case checks with the oracle's own per-step counts that the targeted
path is taken inside at least one call."""
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


def targeted_steps(O, n, L, seed, stream, beta, gamma, chunks):
    """Call-relative steps j >= 3 whose binning is targeted under the rule,
    from the oracle's S and I counts after every step."""
    ref = O.OracleRun(O.SIR, n, L, seed=seed, stream=stream, beta=beta, gamma=gamma)
    counts = []
    for _ in range(sum(chunks)):
        inv = ref.invariants()
        counts.append((inv["n_s"], inv["n_i"]))
        ref.step(1)
    hits, t0 = 0, 0
    for c in chunks:
        for j in range(3, c):
            s, i = counts[t0 + j - 3]     # states at the start of call-relative step j-3
            hits += 32 * s <= i and 10 * i >= n
        t0 += c
    return hits, ref


# (n, L, beta, gamma, chunks)
CASES = [
    (20000, 141, (1, 2), (1, 50), [30, 3, 1, 46]),
    (40000, 200, (1, 3), (1, 80), [80]),
    (5000, 2, (1, 3), (1, 40), [25, 25]),
    (3000, 1, (1, 4), (1, 40), [20, 10]),
    (7000, 3, (1, 3), (1, 60), [40]),
    (100003, 316, (2, 5), (1, 100), [60, 20]),
]


@pytest.mark.parametrize("n,L,beta,gamma,chunks", CASES)
def test_demand_binning_matches_oracle(A, O, n, L, beta, gamma, chunks):
    say(f"case demand binning n={n} L={L} beta={beta} chunks={chunks}")
    hits, ref = targeted_steps(O, n, L, 11, 3, beta, gamma, chunks)
    assert hits > 0, "the workload never reaches the targeted path"
    pop = A.Population(A.SIR, n, L=L, seed=11, stream_id=3, beta=beta, gamma=gamma)
    pop.tune(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_GATHER)
    for c in chunks:
        pop.step(c)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    for g, r in zip(got, ref.columns()):
        assert np.array_equal(g, r)
    assert inv["digest"] == ref.digest()


def test_demand_binning_mixed_with_other_modes(A, O):
    """Gather calls (with the targeted path) alternate with modes that do not
    keep the step counts; the counts must start every gather call at zero."""
    n, L, beta, gamma = 30000, 173, (1, 2), (1, 40)
    chunks = [12, 9, 15, 6, 20, 8]
    tunings = [dict(sir_count=1), dict(sir_count=2), dict(sir_count=1), dict(sir_form=2),
               dict(sir_count=1), dict(sir_count=4)]
    say("case demand binning mixed")
    pop = A.Population(A.SIR, n, L=L, seed=5, stream_id=9, beta=beta, gamma=gamma)
    for c, tu in zip(chunks, tunings):
        pop.tune(**tu)
        pop.step(c)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    ref = O.OracleRun(O.SIR, n, L, seed=5, stream=9, beta=beta, gamma=gamma).step(sum(chunks))
    for g, r in zip(got, ref.columns()):
        assert np.array_equal(g, r)
    assert inv["digest"] == ref.digest()


def test_demand_binning_in_batches(A, O):
    """The same cases stepped together through amber_step_batch (chunked
    into two calls): every run equals the oracle."""
    say("case demand binning batched")
    pops = []
    for k, (n, L, beta, gamma, chunks) in enumerate(CASES):
        p = A.Population(A.SIR, n, L=L, seed=11, stream_id=3 + k, beta=beta, gamma=gamma)
        p.tune(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_GATHER)
        pops.append(p)
    A.step_batch(pops, 37)
    A.step_batch(pops, 23)
    for k, (p, (n, L, beta, gamma, chunks)) in enumerate(zip(pops, CASES)):
        ref = O.OracleRun(O.SIR, n, L, seed=11, stream=3 + k, beta=beta, gamma=gamma).step(60)
        got, inv = p.read(), p.invariants()
        for g, r in zip(got, ref.columns()):
            assert np.array_equal(g, r), (n, L)
        assert inv["digest"] == ref.digest()
        p.release()
