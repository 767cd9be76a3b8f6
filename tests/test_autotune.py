"""Autotuner: host logic on the CPU, invariance and selection on the GPU."""
import json

import pytest

from paper_2601_16292_amd import amber as A
from paper_2601_16292_amd import autotune as T


def test_size_buckets():
    assert T.size_bucket(1) == 0
    assert T.size_bucket(1000) == 9
    assert T.size_bucket(1024) == 10
    assert T.size_bucket(10 ** 6) == 19
    assert T.size_bucket(1 << 27) == 27


def test_candidates_cover_every_knob():
    sir = T.candidates(A.SIR, 10 ** 6, steps=500)
    assert {c.get("sir_count") for c in sir} == {A.COUNT_AUTO, A.COUNT_GATHER, A.COUNT_BOX,
                                                  A.COUNT_EXCHANGE, A.COUNT_TILED,
                                                  A.COUNT_TILED_GATHER, None}
    assert {c.get("sir_form") for c in sir} == {A.SIR_AUTO, A.SIR_PIPELINED, A.SIR_PERSISTENT}
    assert {c.get("sir_poll", 0) for c in sir} == {A.POLL_NOWAIT, A.POLL_PACED}
    # short calls: nothing to pace, and the persistent form can be left out
    short = T.candidates(A.SIR, 10 ** 6, steps=20, persistent=False)
    assert {c.get("sir_poll", 0) for c in short} == {A.POLL_NOWAIT}
    assert A.SIR_PERSISTENT not in {c.get("sir_form") for c in short}
    assert {c.get("wealth_form") for c in T.candidates(A.WEALTH, 10 ** 6)} == \
        {A.WEALTH_ATOMIC, A.WEALTH_EXCHANGE}
    assert all(64 <= c["block"] <= 1024 for c in T.candidates(A.RANDOM_WALK, 10 ** 6))


def test_cache_key_separates_grids_call_lengths_and_sources():
    k = T._key("gfx950:256cu", A.SIR, 10 ** 6, 1000, 500)
    assert k != T._key("gfx950:256cu", A.SIR, 10 ** 6, 4000, 500)      # grid bucket
    assert k != T._key("gfx950:256cu", A.SIR, 10 ** 6, 1000, 100)      # call class
    assert k == T._key("gfx950:256cu", A.SIR, 10 ** 6, 1000, 200)      # same class
    assert k == T._key("gfx950:256cu", A.SIR, 10 ** 6, 0, 500)         # L = round(sqrt N)
    assert f"src={T.source_hash()}" in k
    assert [T.call_class(s) for s in (1, 15, 16, 127, 128)] == [0, 0, 1, 1, 2]


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert T.load_cache(path) == {}
    T.save_cache({"k": {"tuning": {"block": 128}}}, path)
    assert T.load_cache(path) == {"k": {"tuning": {"block": 128}}}
    with open(path, "w") as f:
        f.write("{broken")
    assert T.load_cache(path) == {}


@pytest.mark.gpu
@pytest.mark.parametrize("model,n,L", [(A.SIR, 50000, 223), (A.WEALTH, 100000, 0),
                                       (A.RANDOM_WALK, 100000, 300)])
def test_tuner_picks_a_candidate_with_identical_results(tmp_path, model, n, L):
    import torch
    path = str(tmp_path / "tune.json")
    print(f"case autotune model={model} n={n}", flush=True)
    best = T.tune(model, n, L=L, steps=20, warmup=3, torch=torch, cache_path=path, force=True)
    assert best in T.candidates(model, n, steps=20)
    cache = json.load(open(path))
    (entry,) = cache.values()
    assert len(entry["ms"]) >= 2
    pop = A.Population(model, n, L=L)
    assert T.apply(pop, torch, cache_path=path, steps=20) == best
    st, t = A.amber_get_tuning(pop.handle)
    assert st == A.OK
    pop.release()


@pytest.mark.gpu
def test_tuner_on_long_sir_calls_from_init(tmp_path):
    """Whole runs from the initial state (warmup 0), with the paced and the
    tiled-then-gather candidates: all agree, and the pick is cached under the
    long-call key."""
    import torch
    path = str(tmp_path / "tune.json")
    print("case autotune long SIR calls", flush=True)
    best = T.tune(A.SIR, 40000, L=200, steps=150, warmup=0, torch=torch, cache_path=path,
                  force=True, persistent=False, beta=(1, 3), gamma=(1, 80))
    assert best in T.candidates(A.SIR, 40000, steps=150, persistent=False)
    assert T.lookup(A.SIR, 40000, torch, cache_path=path, L=200, steps=150) == best
    assert T.lookup(A.SIR, 40000, torch, cache_path=path, L=200, steps=50) is None
