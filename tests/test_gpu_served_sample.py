"""The served stream at its stated sizes against the oracle: a stratified
sample of the 10,000-request stream (for each model the first request of
each N decile over [1e4, 1e7], and the model's heaviest request, N near 1e7
and close to 1000 steps) served together as one mix through the continuous
batching loop with its default 50-step chunks, every result checked against
the oracle's stored values (tests/golden/served_sample.json, written by
make_golden.py from the oracle only)."""
import json
import os

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def test_served_sample_matches_oracle(torch):
    from paper_2601_16292_amd import serve, workloads as W
    with open(os.path.join(HERE, "golden", "served_sample.json")) as f:
        gold = {r["id"]: r for r in json.load(f)["runs"]}
    stream = W.served_stream()
    reqs = [dict(stream[i]) for i in sorted(gold)]
    # every request arrives at once (arrival times compressed 1e4 x): they
    # are admitted together and stepped as one mix
    for r in reqs:
        r["arrival"] = r["arrival"] / 1e4
    print(f"case served sample of {len(reqs)} requests, "
          f"{sum(r['n'] * r['steps'] for r in reqs):.3e} agent-steps", flush=True)
    out = serve.serve(reqs, budget_bytes=200 << 30, chunk=50, time_scale=1.0)
    assert out["requests"] == len(reqs)
    assert out["ticks"] > 1
    for rec in out["records"]:
        want = gold[rec["id"]]
        assert (rec["n"], rec["steps"], rec["model"]) == (want["n"], want["steps"], want["model"])
        inv = rec["invariants"]
        assert inv["step"] == want["step"]
        for k in ("digest", "wealth_sum", "wealth_min", "n_s", "n_i", "n_r", "out_of_bounds"):
            assert inv[k] == want[k], (rec["id"], k, inv[k], want[k])
