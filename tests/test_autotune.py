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
    sir = T.candidates(A.SIR, 10 ** 6)
    assert {c.get("sir_count") for c in sir} >= {A.COUNT_GATHER, A.COUNT_BOX}
    assert {c.get("sir_form") for c in sir} == {A.SIR_PIPELINED, A.SIR_PERSISTENT}
    assert {c.get("wealth_form") for c in T.candidates(A.WEALTH, 10 ** 6)} == \
        {A.WEALTH_ATOMIC, A.WEALTH_EXCHANGE}
    assert all(64 <= c["block"] <= 1024 for c in T.candidates(A.RANDOM_WALK, 10 ** 6))


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
    assert best in T.candidates(model, n)
    cache = json.load(open(path))
    (entry,) = cache.values()
    assert len(entry["ms"]) >= 2
    pop = A.Population(model, n, L=L)
    assert T.apply(pop, torch, cache_path=path) == best
    st, t = A.amber_get_tuning(pop.handle)
    assert st == A.OK
    pop.release()
