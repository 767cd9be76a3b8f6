"""GPU parity of the tiled SIR count mode (sir_count = 4): the agents of a call
live as tile-sorted records and every count is binned and summed in LDS.
Results must equal the oracle bit for bit for every tile side, workgroup size,
tile shape (last tile 2 .. T+1 cells wide), occupancy (including every agent
packed into one tile, which takes the several-rounds path) and chunking, and
mixing it with the other modes across calls must not change anything."""
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


def assert_same(pop, ref, steps):
    got = pop.read()
    inv = pop.invariants()
    for g, r in zip(got, ref.columns()):
        assert np.array_equal(g, r)
    assert inv["digest"] == ref.digest() and inv["step"] == steps


# (n, L, tile, chunks, beta, gamma): last tile widths 2, 33, 2, 24, 9, 41
CASES = [
    (3000, 66, 32, [7, 1, 5], (1, 4), (1, 30)),
    (4000, 97, 32, [6, 6], (1, 5), (1, 8)),
    (2500, 130, 64, [9], (1, 3), (1, 30)),
    (8000, 120, 32, [4, 3], (1, 3), (1, 30)),
    (70001, 265, 32, [11, 12], (1, 10), (1, 30)),
    (70001, 265, 64, [23], (1, 10), (1, 30)),
    (200003, 233, 32, [5, 9], (1, 12), (1, 25)),
]


@pytest.mark.parametrize("n,L,tile,chunks,beta,gamma", CASES)
@pytest.mark.parametrize("block", [0, 1024])
def test_tiled_matches_oracle(A, O, n, L, tile, chunks, beta, gamma, block):
    say(f"case tiled n={n} L={L} tile={tile} block={block} chunks={chunks}")
    pop = A.Population(A.SIR, n, L=L, seed=4, stream_id=9, beta=beta, gamma=gamma)
    pop.tune(sir_count=A.COUNT_TILED, sir_tile=tile, **({"block": block} if block else {}))
    for c in chunks:
        pop.step(c)
    ref = O.OracleRun(O.SIR, n, L, seed=4, stream=9, beta=beta, gamma=gamma).step(sum(chunks))
    assert_same(pop, ref, sum(chunks))
    pop.release()


@pytest.mark.parametrize("tile", [32, 64])
def test_tiled_dense_tile(A, O, tile):
    """Every agent starts in one corner tile: one workgroup holds far more
    records than one round of its threads and takes the two-pass path."""
    import torch
    n, L = 30000, 2 * tile + 9
    say(f"case tiled dense corner n={n} L={L} tile={tile}")
    rng = np.random.default_rng(7)
    x = rng.integers(0, 6, n).astype(np.int32)
    y = (L - 1 - rng.integers(0, 5, n)).astype(np.int32)
    s = (rng.random(n) < 0.2).astype(np.uint8)
    pop = A.Population(A.SIR, n, L=L, seed=1, stream_id=2, beta=(1, 40), gamma=(1, 20))
    torch.cuda.synchronize()
    pop.cols[A.COL_X][:n] = torch.from_numpy(x).cuda()
    pop.cols[A.COL_Y][:n] = torch.from_numpy(y).cuda()
    pop.cols[A.COL_STATE][:n] = torch.from_numpy(s).cuda()
    torch.cuda.synchronize()
    pop.tune(sir_count=A.COUNT_TILED, sir_tile=tile, block=64)
    pop.step(6)
    pop.step(5)
    ref = O.OracleRun(O.SIR, n, L, seed=1, stream=2, beta=(1, 40), gamma=(1, 20))
    ref.x[:], ref.y[:], ref.s[:] = x, y, s
    ref.step(11)
    assert_same(pop, ref, 11)
    pop.release()


def test_tiled_mixed_with_other_modes(A, O):
    """Calls alternate between the tiled mode and the grid modes (which expect
    the count grids the tiled mode borrows to be zero again) and forms."""
    n, L = 50000, 223
    chunks = [3, 1, 5, 2, 4, 1, 6, 2]
    tunings = [dict(sir_count=4), dict(sir_count=1), dict(sir_count=4, sir_tile=64),
               dict(sir_count=2), dict(sir_form=2), dict(sir_count=4), dict(sir_count=3),
               dict(sir_count=4, sir_tile=32, block=512)]
    say("case tiled mixed with other modes")
    pop = A.Population(A.SIR, n, L=L, seed=2, stream_id=6, beta=(1, 10), gamma=(1, 30))
    for c, tu in zip(chunks, tunings):
        pop.tune(**tu)
        pop.step(c)
    ref = O.OracleRun(O.SIR, n, L, seed=2, stream=6, beta=(1, 10), gamma=(1, 30)).step(sum(chunks))
    assert_same(pop, ref, sum(chunks))
    pop.release()


def test_tiled_in_batch_uses_grid_mode(A, O):
    say("case tiled runs inside a batch")
    specs = [(20000, 141, 11), (5000, 71, 12), (3000, 0, 13)]
    pops = []
    for n, L, s in specs:
        p = A.Population(A.SIR, n, L=L, seed=0, stream_id=s, beta=(1, 6), gamma=(1, 40))
        p.tune(sir_count=A.COUNT_TILED)
        pops.append(p)
    A.step_batch(pops, 9)
    for p, (n, L, s) in zip(pops, specs):
        ref = O.OracleRun(O.SIR, n, L, seed=0, stream=s, beta=(1, 6), gamma=(1, 40)).step(9)
        assert_same(p, ref, 9)
        p.release()


def test_tiled_unsupported_grid(A):
    pop = A.Population(A.SIR, 4000, L=65, seed=0, stream_id=0)
    pop.tune(sir_count=A.COUNT_TILED)
    with pytest.raises(A.AmberError) as e:
        pop.step(1)
    assert e.value.status == A.E_UNSUPPORTED
    pop.tune(sir_count=A.COUNT_TILED, sir_tile=64)
    with pytest.raises(A.AmberError):
        A.Population(A.SIR, 4000, L=129, seed=0, stream_id=0).tune(
            sir_count=A.COUNT_TILED, sir_tile=64).step(1)
    pop.release()


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "configs.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("tile", [32, 64])
def test_full_sir_1m_tiled(A, golden, tile):
    g = golden["sir_1m"]
    c = g["config"]
    say(f"case full SIR N=1e6 L=1000 x 500 tiled tile={tile}")
    pop = A.Population(A.SIR, c["n"], L=c["L"], seed=c["seed"], stream_id=c["stream"],
                       beta=tuple(c["beta"]), gamma=tuple(c["gamma"]))
    pop.tune(sir_count=A.COUNT_TILED, sir_tile=tile)
    done = 0
    for t in sorted(int(k) for k in g["checkpoints"]):
        pop.step(t - done)
        done = t
        inv = pop.invariants()
        want = g["checkpoints"][str(t)]
        for k in ("digest", "n_s", "n_i", "n_r", "out_of_bounds"):
            assert inv[k] == want[k], (t, k, inv[k], want[k])
    pop.release()


# ------------------------------------------------------------------ tiled, then gather
# (n, L, beta, gamma, initial infected, chunks, sir_poll)
SWITCH_CASES = [
    (40000, 200, (1, 12), (1, 200), 0, [160], 2),          # switch while S > 0
    (40000, 200, (1, 200), (1, 1000), 38900, [120], 2),     # S small from the start
    (40000, 200, (1, 12), (1, 200), 0, [50, 110], 2),       # tiled call, then a switch
    (40000, 200, (1, 12), (1, 200), 0, [160], 1),           # no polls: tiled throughout
    (40000, 200, (1, 12), (1, 200), 0, [50, 110], 0),       # switch only if the count is there
    (40000, 200, (9, 10), (1, 200), 20000, [120], 2),       # no susceptible agent left at the switch
    (40000, 200, (1, 200), (1, 200), 30000, [34], 2),       # one gather step after the switch
]


def expected_tile_bodies(sus, n, chunks, poll):
    """Tiled body launches and switches the host takes: after body i = 16 q
    (q >= 2, i + 1 < steps of the call) it reads the susceptible count summed
    at poll q - 1, which is S after t0 + 16 (q - 1) steps, and ends the tiled
    part after step i once 4 S <= N."""
    bodies = switches = t0 = 0
    for c in chunks:
        k = c
        if poll == 2 and c > 32:
            for q in range(2, c // 16 + 1):
                if 16 * q + 1 >= c:
                    break
                if 4 * sus[t0 + 16 * (q - 1)] <= n:
                    k = 16 * q + 1
                    break
        bodies += k - 1
        switches += k < c
        t0 += c
    return bodies, switches


@pytest.mark.parametrize("n,L,beta,gamma,i0,chunks,poll", SWITCH_CASES)
def test_tiled_then_gather_matches_oracle(A, O, n, L, beta, gamma, i0, chunks, poll):
    say(f"case tiled-then-gather n={n} L={L} beta={beta} i0={i0} chunks={chunks} poll={poll}")
    ref = O.OracleRun(O.SIR, n, L, seed=4, stream=9, beta=beta, gamma=gamma, initial_infected=i0)
    sus = [ref.invariants()["n_s"]]
    for _ in range(sum(chunks)):
        ref.step(1)
        sus.append(ref.invariants()["n_s"])
    bodies, switches = expected_tile_bodies(sus, n, chunks, poll)
    if poll == 2:
        assert switches >= 1
    pop = A.Population(A.SIR, n, L=L, seed=4, stream_id=9, beta=beta, gamma=gamma,
                       initial_infected=i0)
    pop.tune(sir_count=A.COUNT_TILED_GATHER, sir_poll=poll)
    pop.profile(True)
    for c in chunks:
        pop.step(c)
    times = pop.kernel_times()
    if poll == 0:
        # the host switches at a poll whose count the device has already
        # written, or never: at most the paced run's switches, no fewer bodies
        paced_bodies, _ = expected_tile_bodies(sus, n, chunks, 2)
        all_bodies, _ = expected_tile_bodies(sus, n, chunks, 1)
        assert paced_bodies <= times["sir_tile_body"][0] <= all_bodies, times
    else:
        assert times["sir_tile_body"][0] == bodies, (times, bodies)
        # a switch starts a gather segment with its head (a one-step segment
        # has no body launch)
        assert ("sir_head" in times and times["sir_head"][0] > 0) == (switches > 0), times
    assert_same(pop, ref, sum(chunks))
    pop.release()


def test_automatic_modes_on_a_big_grid(A, O):
    """Grids above 16M cells: the automatic choice takes the box mode for a
    call of fewer than 16 steps, the tiled mode up to 127 steps and, from 128
    steps on, the gather mode (tiled then gather when the host may pace the
    call, sir_poll 2); every call must still match the oracle."""
    n, L, beta, gamma = 30000, 4200, (1, 2), (1, 50)
    say(f"case automatic big grid n={n} L={L}")
    pop = A.Population(A.SIR, n, L=L, seed=8, stream_id=1, beta=beta, gamma=gamma)
    pop.profile(True)
    ref = O.OracleRun(O.SIR, n, L, seed=8, stream=1, beta=beta, gamma=gamma)
    done = 0
    for steps, kernel, poll in ((10, "sir_box", 0), (40, "sir_tile_body", 0),
                                (130, "sir_body", 0), (130, "sir_tile_count", 2)):
        pop.tune(sir_poll=poll)
        pop.profile(True)                        # zeroes the per-kernel totals
        pop.step(steps)
        done += steps
        times = pop.kernel_times()
        assert times.get(kernel, (0, 0))[0] > 0, (steps, times)
        ref.step(steps)
        assert_same(pop, ref, done)
    pop.release()
