"""The out-of-cache shapes of the benchmark against the oracle, at their
full size (2^27 agents or rows), in the launch configuration the benchmark
times: the random-walk step (L = 1000, one step per call) and the view
primitives (full and filtered int32 / float32 updates on 2^27-row columns,
an int32 scatter-add of 2^25 entries and a float32 one of 2^22).  Whole
columns are compared bit for bit; inputs are seeded numpy draws."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 1 << 27


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


def _free():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_walk_2p27_one_step_per_call(A, O):
    say("case walk 2^27 L=1000, 3 one-step calls")
    pop = A.Population(A.RANDOM_WALK, N, L=1000, seed=0, stream_id=0)
    for _ in range(3):
        pop.step(1)
    got, inv = pop.read(), pop.invariants()
    pop.release()
    _free()
    ref = O.OracleRun(O.RANDOM_WALK, N, 1000, seed=0, stream=0).step(3)
    for g, r in zip(got, ref.columns()):
        assert np.array_equal(g, r), np.flatnonzero(g != r)[:8]
    assert inv["digest"] == ref.digest() and inv["out_of_bounds"] == 0


def test_views_2p27_rows(A, O):
    import torch
    rng = np.random.default_rng(27)
    col = rng.integers(-1000, 1000, N, dtype=np.int32)
    pred = rng.integers(-5, 6, N, dtype=np.int32)
    say("case view full int32 2^27")
    t = torch.from_numpy(col).cuda()
    A.view_update(t, 3, 1)
    assert np.array_equal(t.cpu().numpy(), O.view_update(col, 3, 1))
    say("case view filtered int32 2^27 (pred > 0)")
    t.copy_(torch.from_numpy(col))
    tp = torch.from_numpy(pred).cuda()
    A.view_update(t, 1, -1, pred=tp, cmp=">", thr=0)
    assert np.array_equal(t.cpu().numpy(), O.view_update(col, 1, -1, pred=pred, cmp=">", thr=0))
    del tp
    say("case scatter-add int32 2^25 entries into 2^27 rows")
    ids = rng.integers(0, N, 1 << 25, dtype=np.int64).astype(np.int32)
    vals = rng.integers(-9, 9, 1 << 25, dtype=np.int32)
    t.copy_(torch.from_numpy(col))
    A.scatter_add(t, torch.from_numpy(ids).cuda(), torch.from_numpy(vals).cuda())
    assert np.array_equal(t.cpu().numpy(), O.scatter_add(col, ids.view(np.uint32), vals))
    del t
    _free()
    say("case view full float32 2^27")
    colf = rng.random(N, dtype=np.float32)
    tf = torch.from_numpy(colf).cuda()
    A.view_update(tf, np.float32(1.5), np.float32(0.25))
    assert np.array_equal(tf.cpu().numpy().view(np.uint32),
                          O.view_update(colf, np.float32(1.5), np.float32(0.25)).view(np.uint32))
    say("case scatter-add float32 2^22 entries into 2^27 rows (list order)")
    m = 1 << 22
    idsf = rng.integers(0, N, m, dtype=np.int64).astype(np.int32)
    idsf[: m // 8] = idsf[0]            # one id hammered: its sum depends on the order
    valsf = rng.standard_normal(m).astype(np.float32)
    tf.copy_(torch.from_numpy(colf))
    A.scatter_add(tf, torch.from_numpy(idsf).cuda(), torch.from_numpy(valsf).cuda())
    want = O.scatter_add(colf, idsf.view(np.uint32), valsf)
    assert np.array_equal(tf.cpu().numpy().view(np.uint32), want.view(np.uint32))
    del tf
    _free()
