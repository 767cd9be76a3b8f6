"""Host logic of the serving loop, on the CPU with a stand-in for the device:
admission by footprint (FIFO, no overtaking), slot limits, chunked stepping
of every resident run, completion records and latency bookkeeping."""
import pytest

from paper_2601_16292_amd import serve


class FakePop:
    live = 0
    peak = 0
    live_bytes = 0
    peak_bytes = 0
    log = []

    def __init__(self, req):
        self.req = req
        self.steps = 0
        FakePop.live += 1
        FakePop.peak = max(FakePop.peak, FakePop.live)
        FakePop.live_bytes += req["bytes"]
        FakePop.peak_bytes = max(FakePop.peak_bytes, FakePop.live_bytes)

    def invariants(self):
        return {"digest": self.req["stream"] * 1000 + self.steps}

    def tune(self, **kw):
        self.tuning = kw

    def step(self, k):
        FakePop.log.append(("alone", k))
        self.steps += k

    def release(self):
        FakePop.live -= 1
        FakePop.live_bytes -= self.req["bytes"]


@pytest.fixture
def fake(monkeypatch):
    FakePop.live = FakePop.peak = FakePop.live_bytes = FakePop.peak_bytes = 0
    FakePop.log = []

    def step_batch(pops, k):
        FakePop.log.append((len(pops), k))
        for p in pops:
            p.steps += k

    monkeypatch.setattr(serve, "_make", FakePop)
    monkeypatch.setattr(serve.A, "step_batch", step_batch)
    monkeypatch.setattr(serve, "footprint", lambda r: r["bytes"])
    return FakePop


def reqs(specs):
    return [dict(stream=i, arrival=a, model=0, n=1000, steps=s, bytes=b)
            for i, (a, s, b) in enumerate(specs)]


def test_every_request_completes_with_its_steps(fake):
    rs = reqs([(0.0, 7, 10), (0.0, 3, 10), (0.0, 12, 10)])
    out = serve.serve(rs, budget_bytes=100, chunk=5, time_scale=1000.0)
    got = {r["id"]: r["digest"] for r in out["records"]}
    assert got == {0: 7, 1: 1003, 2: 2012}     # digest encodes id and steps taken
    assert out["agent_steps"] == 1000 * (7 + 3 + 12)
    batched = [k for w, k in fake.log if w != "alone"]
    assert all(k <= 5 for k in batched)       # batched chunks never exceed the chunk size
    # the last run left alone with nothing queued runs the rest in one call
    assert fake.log[-1] == ("alone", 12 - 5 - 5)


def test_a_lone_run_takes_one_paced_call(fake):
    rs = reqs([(0.0, 40, 10)])
    out = serve.serve(rs, budget_bytes=100, chunk=5, time_scale=1000.0)
    assert fake.log == [("alone", 40)]
    assert out["records"][0]["digest"] == 40


def test_budget_limits_residency_and_keeps_fifo(fake):
    rs = reqs([(0.0, 10, 60), (0.0, 10, 60), (0.0, 2, 10)])
    out = serve.serve(rs, budget_bytes=100, chunk=4, time_scale=1000.0)
    assert fake.peak_bytes <= 100
    recs = {r["id"]: r for r in out["records"]}
    # the 10-byte run fits next to the first one but may not overtake the
    # queued 60-byte run: it is admitted together with it, after run 0 ends
    assert recs[2]["wait_s"] >= recs[1]["wait_s"] > recs[0]["wait_s"]
    assert fake.peak == 2


def test_slot_limit(fake):
    rs = reqs([(0.0, 5, 1)] * 6)
    serve.serve(rs, budget_bytes=100, chunk=5, max_slots=2, time_scale=1000.0)
    assert fake.peak == 2


def test_oversized_request_is_rejected(fake):
    with pytest.raises(ValueError):
        serve.serve(reqs([(0.0, 5, 101)]), budget_bytes=100)


def test_latency_is_measured_from_arrival(fake):
    rs = reqs([(0.0, 3, 1), (0.5, 3, 1)])
    out = serve.serve(rs, budget_bytes=10, chunk=3, time_scale=100.0)
    for r in out["records"]:
        assert r["latency_s"] >= 0 and r["wait_s"] >= 0
    assert out["p99_s"] >= out["p50_s"]
