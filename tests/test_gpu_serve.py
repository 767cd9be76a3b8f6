"""GPU checks of the sweep and serving drivers: results are identical alone,
batched, graph-captured and served in a mix (tolerance 0), and the drivers
report throughput and latency."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def say(*a):
    print(*a, flush=True)


def small_stream(n_requests=40, seed=7):
    from paper_2601_16292_amd import workloads as W
    reqs = W.served_stream(n_requests=n_requests, rate_per_s=50.0, seed=seed, n_lo=1e3,
                           n_hi=2e5, steps_lo=5, steps_hi=60)
    return reqs


def test_served_mix_equals_alone(torch):
    from paper_2601_16292_amd import serve
    reqs = small_stream()
    say(f"case serve {len(reqs)} requests")
    budget = 48 << 20            # small budget: forces queueing and slot reuse
    out = serve.serve([dict(r) for r in reqs], budget_bytes=budget, chunk=7, max_slots=6,
                      time_scale=20.0)
    assert out["requests"] == len(reqs)
    assert out["agent_steps"] == sum(r["n"] * r["steps"] for r in reqs)
    waits = [rec["wait_s"] for rec in out["records"]]
    assert max(waits) > 0                      # some requests had to queue
    by_id = {rec["id"]: rec for rec in out["records"]}
    for r in reqs:
        assert by_id[r["stream"]]["digest"] == serve.alone_digest(r), r["stream"]
    assert out["p99_s"] >= out["p50_s"] > 0


def test_served_digests_match_oracle_sample(torch):
    from oracle import oracle as O
    from paper_2601_16292_amd import serve
    reqs = small_stream(n_requests=12, seed=11)
    out = serve.serve([dict(r) for r in reqs], budget_bytes=1 << 30, chunk=16, time_scale=50.0)
    by_id = {rec["id"]: rec for rec in out["records"]}
    for r in reqs[:6]:
        ref = O.OracleRun(r["model"], r["n"], 0, seed=r["seed"], stream=r["stream"],
                          wealth_init=r.get("wealth_init", 1), beta=r.get("beta", (1, 20)),
                          gamma=r.get("gamma", (1, 100))).step(r["steps"])
        assert by_id[r["stream"]]["digest"] == ref.digest()


def test_plain_server_same_digests(torch):
    from paper_2601_16292_amd import serve
    reqs = small_stream(n_requests=10, seed=3)
    a = serve.serve([dict(r) for r in reqs], budget_bytes=1 << 30, chunk=9, time_scale=50.0)
    b = serve.serve_plain([dict(r) for r in reqs], time_scale=50.0)
    da = {rec["id"]: rec["digest"] for rec in a["records"]}
    db = {rec["id"]: rec["digest"] for rec in b["records"]}
    assert da == db


def test_sweep_forms_identical(torch):
    from paper_2601_16292_amd import sweep, workloads as W
    runs = W.sir_sweep(n_runs=32, steps=20, n_hi=3e4)
    say("case sweep forms, 32 runs")
    plain = sweep.run_plain(runs, torch)
    batched = sweep.run_batched(runs, torch)
    graphed = sweep.run_batched(runs, torch, graph=True)
    assert plain["digests"] == batched["digests"] == graphed["digests"]


def test_graph_replays_match_eager(torch):
    """A captured batched step, replayed several times from a freshly
    initialised state (eager work and syncs in between), equals eager stepping
    every time."""
    from paper_2601_16292_amd import amber as A
    specs = [(A.SIR, 5000 + 333 * i, 40 + i) for i in range(6)] + \
            [(A.WEALTH, 20000, 0), (A.RANDOM_WALK, 7000, 60)]
    eager = []
    for m, n, L in specs:
        p = A.Population(m, n, L=L, seed=1, stream_id=n)
        p.step(11)
        eager.append(p.invariants()["digest"])
        p.release()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pops = [A.Population(m, n, L=L, seed=1, stream_id=n, stream=side) for m, n, L in specs]
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        A.step_batch(pops, 11)
    for rep in range(3):
        if rep:
            # re-initialise the same buffers eagerly, then replay again
            fresh = [A.Population(m, n, L=L, seed=1, stream_id=n, stream=side,
                                  buffers=dict(p.cols, workspace=p.workspace))
                     for p, (m, n, L) in zip(pops, specs)]
            side.synchronize()
        with torch.cuda.stream(side):
            g.replay()
        torch.cuda.synchronize()
        got = [p.invariants()["digest"] for p in pops]   # reads the replayed buffers
        assert got == eager, rep
        if rep:
            for f in fresh:
                f.release()
