"""GPU parity of the gather mode's demand-driven binning: once susceptible
agents are few enough (3 S <= L^2) and infected ones many (10 I >= N),
three steps back, infected agents are binned only on cells a susceptible
agent may read, and once none is left (S = 0, three steps back) nothing is binned
or counted at all.  Every count that is read must still be exact, so
results equal the oracle bit for bit.  Each case checks with the oracle's
own per-step counts that one of the two paths is taken inside a call, and
the cases together take both."""
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
    and those with no susceptible agent left, from the oracle's S and I
    counts after every step."""
    ref = O.OracleRun(O.SIR, n, L, seed=seed, stream=stream, beta=beta, gamma=gamma)
    counts = []
    for _ in range(sum(chunks)):
        inv = ref.invariants()
        counts.append((inv["n_s"], inv["n_i"]))
        ref.step(1)
    targeted, none_left, t0 = 0, 0, 0
    for c in chunks:
        for j in range(3, c):
            s, i = counts[t0 + j - 3]     # states at the start of call-relative step j-3
            targeted += s > 0 and 3 * s <= L * L and 10 * i >= n
            none_left += s == 0
        t0 += c
    return targeted, none_left, ref


# (n, L, beta, gamma, chunks)
CASES = [
    (20000, 141, (1, 2), (1, 50), [30, 3, 1, 46]),
    (40000, 200, (1, 3), (1, 80), [80]),
    (5000, 2, (1, 3), (1, 40), [25, 25]),
    (3000, 1, (1, 4), (1, 40), [20, 10]),
    (7000, 3, (1, 3), (1, 60), [40]),
    (100003, 316, (2, 5), (1, 100), [60, 20]),
    # tiny grids: the marked 3 x 3 blocks wrap onto themselves
    (200, 2, (1, 300), (1, 400), [60]),
    (200, 4, (1, 300), (1, 400), [60]),
    (200, 5, (1, 300), (1, 400), [60]),
]


def test_cases_take_both_paths(O):
    paths = [targeted_steps(O, n, L, 11, 3, b, g, c)[:2] for n, L, b, g, c in CASES]
    assert any(t > 0 for t, _ in paths) and any(z > 0 for _, z in paths)
    # a case that takes both (the 80-step case does so within one call)
    assert any(t > 0 and z > 0 for t, z in paths)


@pytest.mark.parametrize("n,L,beta,gamma,chunks", CASES)
def test_demand_binning_matches_oracle(A, O, n, L, beta, gamma, chunks):
    say(f"case demand binning n={n} L={L} beta={beta} chunks={chunks}")
    targeted, none_left, ref = targeted_steps(O, n, L, 11, 3, beta, gamma, chunks)
    say(f"  targeted steps {targeted}, steps without susceptible agents {none_left}")
    assert targeted + none_left > 0, "the workload never leaves the full binning"
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


@pytest.mark.parametrize("poll", [0, 1, 2])
def test_early_stop_of_a_long_call(A, O, poll):
    """One 200-step call that runs out of susceptible agents near step 40.
    Paced (2), the host stops enqueueing body launches at most 32 launches
    after the one that runs the remaining steps; off (1), every launch is
    enqueued; read-without-waiting (0, the default) stops wherever the host
    first sees the device's word.  All equal the oracle."""
    n, L, beta, gamma, steps = 40000, 200, (1, 3), (1, 80), 200
    say(f"case early stop poll={poll}")
    ref = O.OracleRun(O.SIR, n, L, seed=11, stream=3, beta=beta, gamma=gamma)
    first_none = None
    for t in range(steps):
        if ref.invariants()["n_s"] == 0:
            first_none = t
            break
        ref.step(1)
    assert first_none is not None and first_none + 3 + 2 * 8 < steps - 1
    ref.step(steps - first_none)
    pop = A.Population(A.SIR, n, L=L, seed=11, stream_id=3, beta=beta, gamma=gamma)
    pop.tune(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_GATHER, sir_poll=poll)
    pop.profile(True)
    pop.step(steps)
    body = pop.kernel_times()["sir_body"][0]
    got, inv = pop.read(), pop.invariants()
    pop.release()
    if poll == A.POLL_PACED:
        # the launch running the remaining steps is first_none + 3; polls come
        # every 8 launches, waiting for the launch 8 back
        assert body <= first_none + 3 + 2 * 8, body
    elif poll == A.POLL_OFF:
        assert body == steps - 1
    else:
        assert first_none + 3 <= body <= steps - 1, body
    for g, r in zip(got, ref.columns()):
        assert np.array_equal(g, r)
    assert inv["digest"] == ref.digest()


@pytest.mark.parametrize("poll", [0, 2])
def test_early_stop_in_batches(A, O, poll):
    """Runs that reach the end of their susceptible agents at different steps,
    stepped together in 90-step calls (a run leaves the later launches once
    its remaining steps have run, as soon as the host sees it): every run
    equals the oracle, with the host reading without waiting (0) or paced
    (2)."""
    say(f"case early stop batched poll={poll}")
    specs = [(40000, 200, (1, 3), (1, 80)), (20000, 141, (1, 2), (1, 50)),
             (200, 5, (1, 300), (1, 400)), (30000, 173, (1, 2), (1, 40))]
    pops = []
    for k, (n, L, beta, gamma) in enumerate(specs):
        p = A.Population(A.SIR, n, L=L, seed=7, stream_id=20 + k, beta=beta, gamma=gamma)
        p.tune(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_GATHER, sir_poll=poll)
        pops.append(p)
    A.step_batch(pops, 90)
    A.step_batch(pops, 40)
    for k, (p, (n, L, beta, gamma)) in enumerate(zip(pops, specs)):
        ref = O.OracleRun(O.SIR, n, L, seed=7, stream=20 + k, beta=beta, gamma=gamma).step(130)
        got, inv = p.read(), p.invariants()
        for g, r in zip(got, ref.columns()):
            assert np.array_equal(g, r), (n, L)
        assert inv["digest"] == ref.digest()
        p.release()


@pytest.mark.parametrize("count", ["gather", "tiled_gather"])
def test_captured_long_call_matches_eager(A, count):
    """A 70-step call captured into a graph and replayed on a fresh state
    equals the eager call.  No polling while capturing: in the gather mode
    the launch that finishes the call still runs; the tiled-then-gather mode
    stays tiled, while its eager call may move to the gather mode."""
    import torch
    n, L, beta, gamma = 40000, 200, (1, 3), (1, 80)
    mode = A.COUNT_GATHER if count == "gather" else A.COUNT_TILED_GATHER
    say(f"case captured long call, {count}")
    eager = A.Population(A.SIR, n, L=L, seed=3, stream_id=5, beta=beta, gamma=gamma)
    eager.tune(sir_form=A.SIR_PIPELINED, sir_count=mode)
    eager.step(70)
    want = eager.invariants()["digest"]
    eager.release()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pop = A.Population(A.SIR, n, L=L, seed=3, stream_id=5, beta=beta, gamma=gamma,
                           stream=side)
        pop.tune(sir_form=A.SIR_PIPELINED, sir_count=mode)
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        pop.step(70)
    for rep in range(2):
        fresh = A.Population(A.SIR, n, L=L, seed=3, stream_id=5, beta=beta, gamma=gamma,
                             stream=side, buffers=dict(pop.cols, workspace=pop.workspace))
        side.synchronize()
        with torch.cuda.stream(side):
            g.replay()
        torch.cuda.synchronize()
        assert pop.invariants()["digest"] == want, rep     # reads the replayed buffers
        fresh.release()
    pop.release()


# L = 2049 = 8 * 256 + 1: the wrapped block of a cell in the last column
# spans three coarse columns (the last one a single cell wide)
@pytest.mark.parametrize("n,L,i0", [(200000, 2100, 100000), (150000, 2049, 90000)])
def test_coarse_demand_maps_on_big_grids(A, O, n, L, i0):
    """Grids above 4M cells also keep a coarse demand map (one byte per 8 x 8
    cells; the last block of each axis is partial here) that an infected agent
    reads before its cell's byte.  With half the agents infected from the
    start, the binning is targeted from the fourth launch on; results must
    still equal the oracle."""
    beta, gamma, chunks = (1, 2), (1, 50), [40, 30]
    say(f"case coarse demand maps n={n} L={L} i0={i0}")
    ref = O.OracleRun(O.SIR, n, L, seed=6, stream=2, beta=beta, gamma=gamma, initial_infected=i0)
    inv = ref.invariants()
    assert 3 * inv["n_s"] <= L * L and 10 * inv["n_i"] >= n
    ref.step(sum(chunks))
    assert ref.invariants()["n_s"] < n - i0        # some agents were infected
    pop = A.Population(A.SIR, n, L=L, seed=6, stream_id=2, beta=beta, gamma=gamma,
                       initial_infected=i0)
    pop.tune(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_GATHER)
    for c in chunks:
        pop.step(c)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    for g, r in zip(got, ref.columns()):
        assert np.array_equal(g, r)
    assert inv["digest"] == ref.digest()
