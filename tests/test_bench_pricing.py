"""Host logic of bench.py's roofline pricing (no GPU): algorithmic bytes of
the SIR gather-mode body launches, including the launch that finishes a call
once no susceptible agent is left, and the per-call traffic figure."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_step_bytes(bench):
    n, L = 1000, 40
    assert bench.sir_step_bytes(n, L, 7, 3) == 18 * n + 8 * L * L + 8 * 7
    # no susceptible agent: no count is read, only the columns move
    assert bench.sir_step_bytes(n, L, 7, 0) == 18 * n


def test_gather_body_bytes_one_call_without_finish(bench):
    n, L = 100, 10
    counts = [(50, 5 + k) for k in range(8)]          # S > 0 throughout
    got = bench.sir_gather_body_bytes(n, L, counts, [8])
    want = sum(bench.sir_step_bytes(n, L, i, s) for s, i in counts[1:])
    assert got == want


def test_gather_body_bytes_finishing_launch(bench):
    n, L = 100, 10
    # S reaches 0 at step 2: launch j = 5 (S = 0 three steps back) is the first
    # with F = 2; it costs one column pass and the later launches nothing
    counts = [(9, 1), (4, 5), (0, 8), (0, 8), (0, 7), (0, 6), (0, 6), (0, 5), (0, 5)]
    got = bench.sir_gather_body_bytes(n, L, counts, [9])
    want = sum(bench.sir_step_bytes(n, L, i, s) for s, i in counts[1:5]) + 18 * n
    assert got == want


def test_gather_body_bytes_per_call(bench):
    n, L = 100, 10
    counts = [(0, 3)] * 12
    # two calls of 6: launches 1, 2 (flags 0) priced at the column bytes
    # (S = 0), launch 3 finishes each call
    got = bench.sir_gather_body_bytes(n, L, counts, [6, 6])
    assert got == 2 * (2 * 18 * n + 18 * n)


def test_traffic_per_call_over_this_runs_launches(bench):
    times = {"sir_body": (100, 2.0)}                  # launches, total ms
    priced = {"sir_body": 2_000_000_000}
    traffic = {"sir_body": {"kernel": "sir_body", "bytes_per_call": 3_000_000_000,
                            "launches_per_call": 90}}
    roof = bench.roofline_for(times, priced, traffic)
    assert roof["kernel"] == "sir_body"
    assert roof["traffic"] == 30_000_000
    assert roof["algorithmic_bytes_per_launch"] == 20_000_000
    assert abs(roof["achieved"] - 1000.0) < 1e-6            # 20 MB / 20 us
    assert abs(roof["frac"] - 1000.0 / bench.PEAK_HBM_GBS) < 1e-6
