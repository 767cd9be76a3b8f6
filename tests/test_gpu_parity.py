"""GPU parity: the HIP path through the C ABI against the oracle.

Every comparison is exact (integer arithmetic throughout): whole columns at
sizes the oracle finishes in seconds (several 256-thread tiles and ragged
tails), and digests / invariants / sampled agents against stored oracle
values at the full workload sizes.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


def run_both(A, O, model, n, steps, L=0, seed=0, stream=0, wealth_init=1, beta=(1, 20),
             gamma=(1, 100), i0=0, chunks=None):
    say(f"case model={model} n={n} L={L} steps={steps} seed={seed} stream={stream} "
        f"w0={wealth_init} beta={beta} gamma={gamma} i0={i0} chunks={chunks}")
    pop = A.Population(model, n, L=L, seed=seed, stream_id=stream, wealth_init=wealth_init,
                       beta=beta, gamma=gamma, initial_infected=i0)
    for c in (chunks or [steps]):
        pop.step(c)
    got = pop.read()
    inv = pop.invariants()
    pop.release()
    ref = O.OracleRun(model, n, L, seed=seed, stream=stream, wealth_init=wealth_init, beta=beta,
                      gamma=gamma, initial_infected=i0).step(steps)
    return got, inv, ref


def assert_same(got, inv, ref, steps):
    for g, r in zip(got, ref.columns()):
        if not np.array_equal(g, r):
            bad = np.flatnonzero(g != r)
            raise AssertionError(f"{bad.size} rows differ, first {bad[:8].tolist()}: "
                                 f"gpu {g[bad[:8]].tolist()} oracle {r[bad[:8]].tolist()}")
    ri = ref.invariants()
    assert inv["digest"] == ref.digest()
    assert inv["step"] == steps
    for k in ("wealth_sum", "wealth_min", "n_s", "n_i", "n_r", "out_of_bounds"):
        assert inv[k] == ri[k], k


WALK_CASES = [(1, 1, 5), (2, 2, 9), (3, 3, 4), (5, 7, 20), (63, 10, 7), (64, 1000, 3),
              (65, 5, 11), (1000, 32, 50), (4097, 64, 33), (70001, 265, 12)]


@pytest.mark.parametrize("n,L,steps", WALK_CASES)
def test_walk_parity(A, O, n, L, steps):
    got, inv, ref = run_both(A, O, A.RANDOM_WALK, n, steps, L=L, seed=n, stream=L)
    assert_same(got, inv, ref, steps)


WEALTH_CASES = [(1, 1, 5), (2, 3, 9), (3, 1, 20), (5, 2, 7), (64, 1, 30), (65, 4, 13),
                (1000, 1, 100), (8191, 1, 9), (8192, 2, 6), (8193, 1, 6), (20000, 3, 17),
                (100003, 1, 5)]


@pytest.mark.parametrize("n,w0,steps", WEALTH_CASES)
def test_wealth_parity(A, O, n, w0, steps):
    got, inv, ref = run_both(A, O, A.WEALTH, n, steps, seed=7, stream=n, wealth_init=w0)
    assert_same(got, inv, ref, steps)
    assert inv["wealth_sum"] == n * w0


SIR_CASES = [
    (1, 1, 4, (1, 20), (1, 100), 0), (7, 1, 10, (1, 2), (1, 3), 2),
    (9, 2, 10, (1, 3), (1, 5), 3), (30, 3, 15, (1, 4), (1, 10), 4),
    (65, 4, 12, (1, 20), (1, 100), 5), (1000, 32, 40, (1, 20), (1, 100), 0),
    (5003, 71, 25, (1, 5), (1, 20), 0), (20000, 141, 30, (34, 1500), (1, 100), 50),
    (70001, 265, 20, (300, 1500), (1, 100), 0), (4096, 1000, 10, (999, 1000), (1, 2), 300),
]


@pytest.mark.parametrize("n,L,steps,beta,gamma,i0", SIR_CASES)
def test_sir_parity(A, O, n, L, steps, beta, gamma, i0):
    got, inv, ref = run_both(A, O, A.SIR, n, steps, L=L, seed=3, stream=n, beta=beta,
                             gamma=gamma, i0=i0)
    assert_same(got, inv, ref, steps)
    assert inv["n_s"] + inv["n_i"] + inv["n_r"] == n


@pytest.mark.parametrize("model,n,L", [(0, 5000, 0), (0, 30000, 0), (1, 3001, 50), (2, 6000, 77)])
def test_chunking_invariance(A, O, model, n, L):
    got, inv, ref = run_both(A, O, model, n, 20, L=L, seed=11, stream=2,
                             chunks=[3, 1, 6, 1, 9])
    assert_same(got, inv, ref, 20)


def test_sir_without_transmission_is_the_random_walk(A, O):
    say("case cross-model n=20000 L=150 steps=25")
    sir = A.Population(A.SIR, 20000, L=150, seed=5, stream_id=9, beta=(0, 1), gamma=(0, 1))
    rw = A.Population(A.RANDOM_WALK, 20000, L=150, seed=5, stream_id=9)
    sir.step(25)
    rw.step(25)
    sx, sy, ss = sir.read()
    rx, ry = rw.read()
    assert np.array_equal(sx, rx) and np.array_equal(sy, ry)
    inv = sir.invariants()
    assert inv["n_i"] == 20 and inv["n_r"] == 0 and inv["n_s"] == 20000 - 20


def test_init_state_matches_oracle(A, O):
    for model, n, L in [(0, 777, 0), (1, 100001, 999), (2, 100001, 0)]:
        say(f"case init model={model} n={n} L={L}")
        pop = A.Population(model, n, L=L, seed=9, stream_id=4)
        got = pop.read()
        ref = O.OracleRun(model, n, L, seed=9, stream=4)
        for g, r in zip(got, ref.columns()):
            assert np.array_equal(g, r)
        assert pop.invariants()["step"] == 0
        assert pop.info().grid_side == ref.L


# ------------------------------------------------------------------ full sizes

@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "configs.json")) as f:
        return json.load(f)


def test_full_wealth_1k(A, golden):
    g = golden["wealth_1k"]
    c = g["config"]
    say("case full wealth N=1000 x 100")
    pop = A.Population(A.WEALTH, c["n"], seed=c["seed"], stream_id=c["stream"],
                       wealth_init=c["wealth_init"])
    done = 0
    for t in sorted(int(k) for k in g["checkpoints"]):
        pop.step(t - done)
        done = t
        inv = pop.invariants()
        want = g["checkpoints"][str(t)]
        assert inv["digest"] == want["digest"] and inv["wealth_sum"] == want["wealth_sum"]
    (w,) = pop.read()
    assert w.tolist() == g["wealth"]


def test_full_walk_1m(A, O, golden):
    g = golden["walk_1m"]
    c = g["config"]
    say("case full random walk N=1e6 L=1000 x 1000")
    pop = A.Population(A.RANDOM_WALK, c["n"], L=c["L"], seed=c["seed"], stream_id=c["stream"])
    done = 0
    for t in sorted(int(k) for k in g["checkpoints"]):
        pop.step(t - done)
        done = t
        inv = pop.invariants()
        want = g["checkpoints"][str(t)]
        assert inv["digest"] == want["digest"], t
        assert inv["out_of_bounds"] == 0
    x, y = pop.read()
    ids = np.array(g["sample_ids"])
    assert x[ids].tolist() == g["sample_x"] and y[ids].tolist() == g["sample_y"]
    # a few more agents replayed alone by the oracle
    more = np.array([0, 1, 2, 3, 999_999, 500_000, 123_457], dtype=np.uint32)
    ox, oy = O.walk_agents(more, c["L"], c["seed"], c["stream"], c["steps"])
    assert np.array_equal(x[more], ox) and np.array_equal(y[more], oy)


@pytest.mark.parametrize("form,count", [(1, 1), (1, 2), (1, 3), (2, 0)])
def test_full_sir_1m(A, golden, form, count):
    g = golden["sir_1m"]
    c = g["config"]
    say(f"case full SIR N=1e6 L=1000 x 500 form={form} count={count}")
    pop = A.Population(A.SIR, c["n"], L=c["L"], seed=c["seed"], stream_id=c["stream"],
                       beta=tuple(c["beta"]), gamma=tuple(c["gamma"]))
    pop.tune(sir_form=form, sir_count=count)
    done = 0
    for t in sorted(int(k) for k in g["checkpoints"]):
        pop.step(t - done)
        done = t
        inv = pop.invariants()
        want = g["checkpoints"][str(t)]
        for k in ("digest", "n_s", "n_i", "n_r", "out_of_bounds"):
            assert inv[k] == want[k], (t, k, inv[k], want[k])


# ------------------------------------------------------------------ error paths on device

def test_device_validation(A):
    import torch
    say("case device validation")
    d = A.make_desc(A.RANDOM_WALK, 1000, 10)
    ws = torch.empty(A.amber_workspace_bytes(d), dtype=torch.uint8, device="cuda")
    x = torch.empty(A.amber_column_bytes(d, A.COL_X) // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    host = np.zeros(2000, dtype=np.int32)
    b = A.Buffers()
    b.col[A.COL_X], b.col[A.COL_Y] = x.data_ptr(), host.ctypes.data
    b.workspace, b.workspace_bytes = ws.data_ptr(), ws.numel()
    st, h = A.amber_init_population(d, b, 0)
    assert st == A.E_INVALID and "device" in A.amber_last_error()
    b.col[A.COL_Y] = y.data_ptr() + 4
    st, h = A.amber_init_population(d, b, 0)
    assert st == A.E_INVALID and "aligned" in A.amber_last_error()
    b.col[A.COL_Y] = y.data_ptr()
    b.workspace_bytes = 8
    st, h = A.amber_init_population(d, b, 0)
    assert st == A.E_NOMEM
    b.workspace_bytes = ws.numel()
    st, h = A.amber_init_population(d, b, 0)
    assert st == A.OK
    assert A.amber_release(h) == A.OK
    assert A.amber_release(h) == A.E_STATE
    assert A.amber_step(h, 1) == A.E_STATE


def _allocation_range(ptr):
    """(base, size) of the HIP allocation holding device address ptr, or None."""
    import ctypes
    try:
        hip = ctypes.CDLL("libamdhip64.so")
    except OSError:
        return None
    base, size = ctypes.c_void_p(), ctypes.c_size_t()
    if hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), ctypes.c_void_p(ptr)) != 0:
        return None
    return base.value, size.value


def test_buffers_shorter_than_their_allocation_allows(A):
    """A buffer that starts too close to the end of its allocation is refused.
    Each case also carries a later fault (a host workspace, a workspace off the
    256-byte grid), so that nothing is enqueued even if the extent check were
    missing: only the error message tells which check fired."""
    import torch
    say("case buffer extent")
    d = A.make_desc(A.RANDOM_WALK, 1000, 10)
    need = A.amber_column_bytes(d, A.COL_X)
    x = torch.empty(need // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    ws = torch.empty(A.amber_workspace_bytes(d) + 512, dtype=torch.uint8, device="cuda")
    rng = _allocation_range(y.data_ptr())
    if rng is None:
        pytest.skip("the runtime does not report allocation extents")
    base, size = rng
    assert base <= y.data_ptr() and y.data_ptr() + need <= base + size
    host_ws = np.zeros(64, dtype=np.uint8)
    b = A.Buffers()
    b.col[A.COL_X], b.col[A.COL_Y] = x.data_ptr(), (base + size - 256) & ~15
    b.workspace, b.workspace_bytes = host_ws.ctypes.data, A.amber_workspace_bytes(d)
    st, h = A.amber_init_population(d, b, 0)
    assert st == A.E_INVALID and "y column" in A.amber_last_error() \
        and "allocation" in A.amber_last_error(), A.amber_last_error()
    b.col[A.COL_Y] = y.data_ptr()
    wbase, wsize = _allocation_range(ws.data_ptr())
    b.workspace = ((wbase + wsize - A.amber_workspace_bytes(d) // 2) & ~255) + 16
    st, h = A.amber_init_population(d, b, 0)
    assert st == A.E_INVALID and "workspace" in A.amber_last_error() \
        and "allocation" in A.amber_last_error(), A.amber_last_error()
    b.workspace = ws.data_ptr()
    st, h = A.amber_init_population(d, b, 0)
    assert st == A.OK, A.amber_last_error()
    assert A.amber_release(h) == A.OK


# ------------------------------------------------------------------ launch shapes

def _sir_tuned(A, n, L, steps, chunks, tunings, seed=2, stream=6, beta=(1, 10), gamma=(1, 30)):
    pop = A.Population(A.SIR, n, L=L, seed=seed, stream_id=stream, beta=beta, gamma=gamma)
    for c, tu in zip(chunks, tunings):
        pop.tune(**tu)
        pop.step(c)
    got = pop.read()
    inv = pop.invariants()
    pop.release()
    return got, inv


SIR_FORMS = [dict(sir_form=1), dict(sir_form=1, block=64), dict(sir_form=1, block=1024),
             dict(sir_form=1, sir_count=1), dict(sir_form=1, sir_count=2),
             dict(sir_form=1, sir_count=2, block=128), dict(sir_form=1, sir_count=3),
             dict(sir_form=2, max_groups_per_thread=1), dict(sir_form=2, max_groups_per_thread=2),
             dict(sir_form=2, max_groups_per_thread=8), dict(sir_form=0)]


@pytest.mark.parametrize("n,L", [(1, 1), (7, 2), (4097, 64), (70001, 265)])
@pytest.mark.parametrize("tu", SIR_FORMS)
def test_sir_launch_forms_match_oracle(A, O, n, L, tu):
    say(f"case sir form {tu} n={n} L={L}")
    try:
        got, inv = _sir_tuned(A, n, L, 23, [23], [tu])
    except A.AmberError as e:
        if e.status == A.E_UNSUPPORTED and tu.get("sir_count") == 3 and L < 12:
            pytest.skip("exchange mode needs at least 3 bands (grid side >= 3)")
        raise
    ref = O.OracleRun(O.SIR, n, L, seed=2, stream=6, beta=(1, 10), gamma=(1, 30)).step(23)
    assert_same(got, inv, ref, 23)


def test_sir_forms_mixed_across_calls(A, O):
    n, L = 50000, 223
    chunks = [1, 5, 1, 7, 2, 1, 9, 1, 4, 3]
    tunings = [dict(sir_form=2), dict(sir_form=1), dict(sir_form=1, sir_count=2), dict(sir_form=2),
               dict(sir_form=1, block=128), dict(sir_form=2, max_groups_per_thread=4),
               dict(sir_form=0), dict(sir_count=3), dict(sir_count=1), dict(sir_count=2)]
    say("case sir mixed forms")
    got, inv = _sir_tuned(A, n, L, sum(chunks), chunks, tunings)
    ref = O.OracleRun(O.SIR, n, L, seed=2, stream=6, beta=(1, 10), gamma=(1, 30)).step(sum(chunks))
    assert_same(got, inv, ref, sum(chunks))


@pytest.mark.parametrize("model,n", [(0, 30001), (1, 30001)])
@pytest.mark.parametrize("block", [64, 192, 1024])
def test_block_size_invariance(A, O, model, n, block):
    say(f"case block={block} model={model}")
    pop = A.Population(model, n, L=97, seed=1, stream_id=3)
    pop.tune(block=block)
    pop.step(13)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    ref = O.OracleRun(model, n, 97, seed=1, stream=3).step(13)
    assert_same(got, inv, ref, 13)


def test_tuning_validation(A):
    pop = A.Population(A.RANDOM_WALK, 100, L=10)
    for bad in [dict(block=32), dict(block=1088), dict(block=100), dict(sir_form=3),
                dict(max_groups_per_thread=3), dict(sir_count=6), dict(wealth_form=4),
                dict(sir_tile=16), dict(sir_tile=48), dict(sir_poll=3)]:
        with pytest.raises(A.AmberError):
            pop.tune(**bad)
    st, t = A.amber_get_tuning(pop.handle)
    assert st == A.OK and t.block == 256
    pop.release()


@pytest.mark.parametrize("n,w0,steps", [(8193, 1, 7), (12305, 3, 5), (100003, 1, 6),
                                        (1 << 20, 1, 4), ((1 << 21) + 5, 1, 3)])
@pytest.mark.parametrize("form", [1, 2])
def test_wealth_forms_match_oracle(A, O, n, w0, steps, form):
    say(f"case wealth form={form} n={n} w0={w0} steps={steps}")
    pop = A.Population(A.WEALTH, n, seed=5, stream_id=n, wealth_init=w0)
    pop.tune(wealth_form=form)
    pop.step(steps)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    ref = O.OracleRun(O.WEALTH, n, seed=5, stream=n, wealth_init=w0).step(steps)
    assert_same(got, inv, ref, steps)


@pytest.mark.parametrize("n,w0,steps,chunks,form", [((1 << 24) + 12345, 1, 3, [3], 2),
                                                    ((1 << 25) + 7, 2, 4, [1, 3], 2),
                                                    (40_000_001, 1, 3, [2, 1], 2),
                                                    ((5 << 23) + 1, 1, 2, [2], 2),
                                                    (5 << 23, 2, 2, [2], 2),
                                                    (1 << 27, 1, 3, [2, 1], 2),
                                                    ((1 << 24) + 12345, 1, 3, [1, 2], 3),
                                                    ((5 << 23) + 1, 3, 3, [3], 3)])
def test_wealth_exchange_above_2p24(A, O, n, w0, steps, chunks, form):
    """Partitions of 2^15 agents (up to 5 * 2^23 agents) and 2^16 agents (above),
    16-bit records, ragged last partitions, both kernels at their most
    partitions (5 * 2^23 and 2^27 agents, the benchmarked size), the
    fold-only call boundary; form
    3 folds every partition with the 32-bit two-pass counters that a 16-bit
    counter's wrap would call for."""
    say(f"case wealth exchange 16-bit kernels n={n} chunks={chunks} form={form}")
    pop = A.Population(A.WEALTH, n, seed=3, stream_id=7, wealth_init=w0)
    pop.tune(wealth_form=form)
    for c in chunks:
        pop.step(c)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    ref = O.OracleRun(O.WEALTH, n, seed=3, stream=7, wealth_init=w0).step(steps)
    assert_same(got, inv, ref, steps)


def test_wealth_forms_mixed_across_calls(A, O):
    n = 300007
    chunks = [1, 3, 1, 2, 5, 1]
    forms = [2, 1, 2, 2, 1, 0]
    say("case wealth mixed forms")
    pop = A.Population(A.WEALTH, n, seed=8, stream_id=1, wealth_init=2)
    for c, f in zip(chunks, forms):
        pop.tune(wealth_form=f)
        pop.step(c)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    ref = O.OracleRun(O.WEALTH, n, seed=8, stream=1, wealth_init=2).step(sum(chunks))
    assert_same(got, inv, ref, sum(chunks))
