"""GPU parity of the batched form (amber_step_batch): every run of a batch must
equal the same run stepped alone and the oracle, bit for bit, whatever the mix
of models, sizes, step indices and chunking of runs into launches."""
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


def make(A, spec):
    return A.Population(spec["model"], spec["n"], L=spec.get("L", 0), seed=spec.get("seed", 0),
                        stream_id=spec["stream"], wealth_init=spec.get("w0", 1),
                        beta=spec.get("beta", (1, 20)), gamma=spec.get("gamma", (1, 100)))


def oracle_run(O, spec, steps):
    return O.OracleRun(spec["model"], spec["n"], spec.get("L", 0), seed=spec.get("seed", 0),
                       stream=spec["stream"], wealth_init=spec.get("w0", 1),
                       beta=spec.get("beta", (1, 20)), gamma=spec.get("gamma", (1, 100))).step(steps)


MIX = [
    dict(model=0, n=1, stream=1), dict(model=0, n=777, stream=2, w0=3),
    dict(model=0, n=8192, stream=3), dict(model=0, n=8193, stream=4),
    dict(model=0, n=50001, stream=5, w0=2),
    dict(model=1, n=1, L=1, stream=6), dict(model=1, n=999, L=31, stream=7),
    dict(model=1, n=100003, L=300, stream=8),
    dict(model=2, n=1, L=1, stream=9), dict(model=2, n=13, L=2, stream=10, beta=(1, 2)),
    dict(model=2, n=1000, L=32, stream=11, beta=(34, 1500)),
    dict(model=2, n=60001, L=0, stream=12, beta=(1, 5), gamma=(1, 20)),
]


def test_mixed_batch_matches_oracle(A, O):
    say("case mixed batch")
    pops = [make(A, s) for s in MIX]
    # uneven step indices: some runs step alone first
    pre = [i % 3 for i in range(len(MIX))]
    for p, k in zip(pops, pre):
        if k:
            p.step(k)
    A.step_batch(pops, 9)
    A.step_batch(pops, 1)
    A.step_batch(pops[::2], 4)
    for i, (p, spec) in enumerate(zip(pops, MIX)):
        steps = pre[i] + 10 + (4 if i % 2 == 0 else 0)
        got = p.read()
        inv = p.invariants()
        ref = oracle_run(O, spec, steps)
        for g, r in zip(got, ref.columns()):
            assert np.array_equal(g, r), (i, spec)
        assert inv["digest"] == ref.digest() and inv["step"] == steps
        p.release()


@pytest.mark.parametrize("count", [1, 2, 3, "mixed"])
def test_many_runs_chunked_into_launches(A, O, count):
    say(f"case 53 SIR runs in one batch, count mode {count}")
    specs = [dict(model=2, n=100 + 37 * i, L=0, stream=100 + i,
                  beta=((15 + 19 * (i % 16)), 1500)) for i in range(53)]
    pops = [make(A, s) for s in specs]
    for i, p in enumerate(pops):
        # mixed: every count mode, the tiled ones (4, 5) mapped by the batch
        # to the automatic mode where their tiles fit
        p.tune(sir_count=(1 + i % 5) if count == "mixed" else count)
    A.step_batch(pops, 17)
    for p, s in zip(pops, specs):
        ref = oracle_run(O, s, 17)
        assert p.invariants()["digest"] == ref.digest()
        p.release()


def test_batch_equals_alone(A):
    say("case batch == alone, 40 walk + 40 wealth runs")
    specs = ([dict(model=1, n=3000 + 11 * i, L=50 + i, stream=i) for i in range(40)] +
             [dict(model=0, n=9000 + 101 * i, stream=50 + i) for i in range(40)])
    batch = [make(A, s) for s in specs]
    alone = [make(A, s) for s in specs]
    A.step_batch(batch, 12)
    for p in alone:
        p.step(12)
    for b, a in zip(batch, alone):
        assert b.invariants()["digest"] == a.invariants()["digest"]
        for cb, ca in zip(b.read(), a.read()):
            assert np.array_equal(cb, ca)
        b.release()
        a.release()


def test_batch_errors(A):
    p = make(A, dict(model=1, n=100, L=10, stream=0))
    with pytest.raises(A.AmberError):
        A.step_batch([p, p], 1)
    assert A.amber_step_batch([p.handle], 0) == A.OK
    p.release()


@pytest.fixture(scope="module")
def sweep_golden():
    path = os.path.join(HERE, "golden", "sweep.json")
    if not os.path.exists(path):
        pytest.skip("sweep golden values not generated")
    with open(path) as f:
        return json.load(f)


def test_full_sir_sweep_batched(A, sweep_golden):
    """The 256-replicate SIR sweep (N log-uniform in [1e3, 1e6], 16 betas,
    300 steps) stepped as one batch equals the oracle replicate by replicate."""
    from paper_2601_16292_amd import workloads as W
    runs = W.sir_sweep()
    say(f"case full sweep, {len(runs)} runs, sum N = {sum(r['n'] for r in runs)}")
    pops = [A.Population(A.SIR, r["n"], L=r["L"], seed=r["seed"], stream_id=r["stream"],
                         beta=r["beta"], gamma=r["gamma"]) for r in runs]
    for i, p in enumerate(pops):
        p.tune(sir_count=1 + (i % 3))       # every count mode inside one sweep
    A.step_batch(pops, sweep_golden["steps"])
    for p, want in zip(pops, sweep_golden["runs"]):
        inv = p.invariants()
        for k in ("digest", "n_s", "n_i", "n_r", "step"):
            assert inv[k] == want[k], (want["stream"], k)
        p.release()


def test_wealth_batch_forms_match_oracle(A, O):
    """Large wealth runs in one batch, some on the atomic path and some on the
    partition exchange (both partition sizes), at uneven step indices."""
    say("case wealth batch forms")
    specs = [dict(model=0, n=n, stream=200 + i, w0=1 + i % 3)
             for i, n in enumerate([9001, 20000, 65537, 300001, (1 << 21) + 77, 12345, 40000])]
    pops = [make(A, s) for s in specs]
    for i, p in enumerate(pops):
        p.tune(wealth_form=1 if i % 3 == 1 else 0)
        if i % 2:
            p.step(2)
    A.step_batch(pops, 5)
    for i, (p, s) in enumerate(zip(pops, specs)):
        steps = 5 + (2 if i % 2 else 0)
        ref = oracle_run(O, s, steps)
        (w,) = p.read()
        assert np.array_equal(w, ref.w), (i, s)
        p.release()
