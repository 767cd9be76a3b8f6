"""The per-kernel timer (amber_profile_enable / amber_profile_read): launch
counts per kernel, positive times, totals cleared on enable, and results
identical with and without timing."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2601_16292_amd import amber
    amber.lib()
    return amber


def run(A, model, n, L, steps, calls, profile, **tuning):
    p = A.Population(model, n, L=L, seed=3, stream_id=1)
    if tuning:
        p.tune(**tuning)
    if profile:
        p.profile(True)
    for _ in range(calls):
        p.step(steps)
    t = p.kernel_times() if profile else None
    d = p.invariants()["digest"]
    p.release()
    return t, d


def test_sir_pipelined_counts(A):
    print("case profile SIR pipelined", flush=True)
    t, d = run(A, A.SIR, 20000, 0, 10, 2, True, sir_form=A.SIR_PIPELINED,
               sir_count=A.COUNT_GATHER)
    assert t["sir_head"][0] == 2 and t["sir_tail"][0] == 2 and t["sir_clear"][0] == 2
    assert t["sir_body"][0] == 18          # 9 per call, timed back to back
    assert all(ms > 0 for _, ms in t.values())
    _, d0 = run(A, A.SIR, 20000, 0, 10, 2, False, sir_form=A.SIR_PIPELINED,
                sir_count=A.COUNT_GATHER)
    assert d == d0


def test_sir_box_alternating_counts(A):
    print("case profile SIR box", flush=True)
    t, d = run(A, A.SIR, 20000, 0, 7, 1, True, sir_count=A.COUNT_BOX)
    assert t["sir_box"][0] == 7 and t["sir_body_box"][0] == 6
    _, d0 = run(A, A.SIR, 20000, 0, 7, 1, False, sir_count=A.COUNT_BOX)
    assert d == d0


def test_wealth_atomic_counts(A):
    print("case profile wealth atomic", flush=True)
    t, d = run(A, A.WEALTH, 100000, 0, 5, 3, True, wealth_form=A.WEALTH_ATOMIC)
    assert t["wealth_step"][0] == 15 and t["wealth_fold"][0] == 3
    _, d0 = run(A, A.WEALTH, 100000, 0, 5, 3, False, wealth_form=A.WEALTH_ATOMIC)
    assert d == d0


def test_enable_clears_totals(A):
    print("case profile clear", flush=True)
    p = A.Population(A.RANDOM_WALK, 5000, L=70, seed=0, stream_id=0)
    p.profile(True)
    p.step(4)
    p.step(4)
    assert p.kernel_times()["walk"][0] == 2  # one launch per call
    p.profile(True)
    p.step(1)
    assert p.kernel_times()["walk"][0] == 1
    p.release()
