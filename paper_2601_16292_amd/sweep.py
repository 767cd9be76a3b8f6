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
on the host).  The batched form runs the replicates in a few waves, smallest
first, so that small replicates complete early.
"""
import time

import numpy as np

from . import amber as A


def _percentiles(lat):
    lat = np.asarray(lat, dtype=np.float64)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def _make(run, stream=None, buffers=None):
    return A.Population(A.SIR, run["n"], L=run["L"], seed=run["seed"], stream_id=run["stream"],
                        beta=run["beta"], gamma=run["gamma"], stream=stream, buffers=buffers)


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


def run_batched(runs, torch, graph=False, waves=4):
    """The replicates in `waves` batches of about equal size, smallest runs
    first (shortest-job-first: the small replicates complete early), each
    batch one amber_step_batch call; a replicate's latency is taken when its
    batch's invariants are on the host.  With graph=True each wave's batched
    step launches are captured into a graph first (state initialised outside
    it) and replayed: the capture time is reported apart (capture_s) and is
    not part of the timed sweep."""
    steps = runs[0]["steps"]
    assert all(r["steps"] == steps for r in runs)
    order = sorted(range(len(runs)), key=lambda i: (runs[i]["n"], i))
    k = max(1, min(waves, len(runs)))
    parts = [order[w * len(order) // k:(w + 1) * len(order) // k] for w in range(k)]
    lat = [0.0] * len(runs)
    digests = [0] * len(runs)
    work = sum(r["n"] * r["steps"] for r in runs)
    capture_s = setup_s = 0.0
    torch.cuda.synchronize()
    if graph:
        # capture every wave on a side stream before the clock starts
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        staged = []
        c0 = time.perf_counter()
        for part in parts:
            with torch.cuda.stream(side):
                pops = [_make(runs[i], stream=side) for i in part]
            side.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                A.step_batch(pops, steps)
            staged.append((part, pops, g))
        capture_s = time.perf_counter() - c0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for part, pops, g in staged:
            # initial states written again into the captured buffers (as the
            # other forms create theirs inside the clock), then one replay
            s0 = time.perf_counter()
            with torch.cuda.stream(side):
                fresh = [_make(runs[i], stream=side,
                               buffers=dict(p.cols, workspace=p.workspace))
                         for i, p in zip(part, pops)]
            setup_s += time.perf_counter() - s0
            with torch.cuda.stream(side):
                g.replay()
            for i, p in zip(part, pops):
                inv = p.invariants()
                digests[i] = inv["digest"]
            now = time.perf_counter() - t0
            for i in part:
                lat[i] = now
            for q in fresh:
                q.release()
        secs = time.perf_counter() - t0
        for _, pops, _ in staged:
            for p in pops:
                p.release()
    else:
        t0 = time.perf_counter()
        for part in parts:
            s0 = time.perf_counter()
            pops = [_make(runs[i]) for i in part]
            setup_s += time.perf_counter() - s0
            A.step_batch(pops, steps)
            for i, p in zip(part, pops):
                digests[i] = p.invariants()["digest"]
            now = time.perf_counter() - t0
            for i in part:
                lat[i] = now
            for p in pops:
                p.release()
        secs = time.perf_counter() - t0
    p50, p99 = _percentiles(lat)
    return dict(seconds=secs, agent_steps=work, value=work / secs, p50_s=p50, p99_s=p99,
                digests=digests, setup_s=setup_s, capture_s=capture_s,
                order=f"{k} waves, smallest replicates first")
