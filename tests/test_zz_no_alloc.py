"""The no-allocation entry point (amber_init_population_noalloc) against the
ordinary one: same descriptor, same columns and invariants after the same
steps, on two calls in a row per case, the second with a smaller input (the
device scratch then holds the first run's contents, which init must clear
where the run needs zeros).  Also the exclusive use of the scratch, and the
size limit."""
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


def say(*a):
    print(*a, flush=True)


def _run(A, model, n, L, steps, chunks, tuning, noalloc, **kw):
    pop = A.Population(model, n, L=L, seed=5, stream_id=n % 97, noalloc=noalloc, **kw)
    if tuning:
        pop.tune(**tuning)
    done = 0
    for c in chunks:
        pop.step(c)
        done += c
    assert done == steps
    got, inv = pop.read(), pop.invariants()
    pop.release()
    return got, inv


# (model, [(n, L), (smaller n, L)], steps split into calls, tuning)
CASES = [
    (2, [(300000, 548), (50000, 224)], [7, 33], dict(sir_count=1)),
    (2, [(250000, 500), (20011, 141)], [40], dict(sir_count=4, sir_tile=32)),
    (2, [(90000, 300), (4097, 64)], [25], dict(sir_form=2)),
    (0, [(1000000, 0), (100003, 0)], [3, 4], dict(wealth_form=2)),
    (0, [(500000, 0), (8193, 0)], [5], dict(wealth_form=1)),
    (0, [(5000, 0), (1000, 0)], [100], {}),
    (1, [(1000000, 1000), (70001, 265)], [50], {}),
]


@pytest.mark.parametrize("model,sizes,chunks,tuning", CASES)
def test_noalloc_equals_ordinary_on_two_calls(A, model, sizes, chunks, tuning):
    steps = sum(chunks)
    for n, L in sizes:
        say(f"case noalloc model={model} n={n} L={L} chunks={chunks} tuning={tuning}")
        ref = _run(A, model, n, L, steps, chunks, tuning, noalloc=False)
        got = _run(A, model, n, L, steps, chunks, tuning, noalloc=True)
        for g, r in zip(got[0], ref[0]):
            assert np.array_equal(g, r), (model, n)
        for k in ("digest", "step", "wealth_sum", "wealth_min", "n_s", "n_i", "n_r",
                  "out_of_bounds"):
            assert got[1][k] == ref[1][k], (model, n, k)


def test_noalloc_scratch_is_exclusive_and_bounded(A):
    say("case noalloc exclusive and bounded")
    first = A.Population(A.RANDOM_WALK, 1000, L=30, noalloc=True)
    with pytest.raises(A.AmberError) as e:
        A.Population(A.RANDOM_WALK, 1000, L=30, noalloc=True)
    assert e.value.status == A.E_STATE
    first.release()
    second = A.Population(A.RANDOM_WALK, 1000, L=30, noalloc=True)   # free again
    second.step(3)
    assert second.invariants()["out_of_bounds"] == 0
    second.release()
    with pytest.raises(A.AmberError) as e:
        A.Population(A.SIR, 2_000_000, noalloc=True)                 # workspace above 32 MiB
    assert e.value.status == A.E_UNSUPPORTED
