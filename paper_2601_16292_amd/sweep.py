"""Parameter sweep driver: many SIR replicates advanced by the GPU library.

The sweep is the experiment layer of the method (parameter points x
replicates, Sec. 4.2) executed on one GPU.  Two execution forms with identical
results:

  plain    each replicate alone: init, then amber_step(steps) on one stream,
           replicate after replicate (one launch per step per replicate);
  batched  all replicates initialised, then amber_step_batch over all of them
           (one launch per step per chunk of replicates), optionally captured
           once into a HIP graph by the caller's stream capture and replayed.

Both report aggregate agent-steps/s and per-replicate completion latency
(p50/p99, measured from sweep submission to the replicate's invariants being
on the host).
"""
import time

import numpy as np

from . import amber as A


def _percentiles(lat):
    lat = np.asarray(lat, dtype=np.float64)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def _make(run, stream=None):
    return A.Population(A.SIR, run["n"], L=run["L"], seed=run["seed"], stream_id=run["stream"],
                        beta=run["beta"], gamma=run["gamma"], stream=stream)


def run_plain(runs, torch):
    """Replicate after replicate; latency of replicate i = time from sweep
    start until its invariants are read back."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, digests, work = [], [], 0
    for r in runs:
        p = _make(r)
        p.step(r["steps"])
        inv = p.invariants()
        lat.append(time.perf_counter() - t0)
        digests.append(inv["digest"])
        work += r["n"] * r["steps"]
        p.release()
    secs = time.perf_counter() - t0
    p50, p99 = _percentiles(lat)
    return dict(seconds=secs, agent_steps=work, value=work / secs, p50_s=p50, p99_s=p99,
                digests=digests)


def run_batched(runs, torch, graph=False):
    """All replicates in one batch.  With graph=True the batched step launches
    are captured into a graph first (state initialised outside it) and the
    graph is replayed once."""
    steps = runs[0]["steps"]
    assert all(r["steps"] == steps for r in runs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            pops = [_make(r, stream=side) for r in runs]
        side.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            A.step_batch(pops, steps)
        with torch.cuda.stream(side):
            g.replay()
        torch.cuda.synchronize()
    else:
        pops = [_make(r) for r in runs]
        A.step_batch(pops, steps)
    lat, digests, work = [], [], 0
    for r, p in zip(runs, pops):
        inv = p.invariants()
        lat.append(time.perf_counter() - t0)
        digests.append(inv["digest"])
        work += r["n"] * r["steps"]
    secs = time.perf_counter() - t0
    for p in pops:
        p.release()
    p50, p99 = _percentiles(lat)
    return dict(seconds=secs, agent_steps=work, value=work / secs, p50_s=p50, p99_s=p99,
                digests=digests)
