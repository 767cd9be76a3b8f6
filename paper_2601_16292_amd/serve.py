"""Serving loop: simulation runs arrive over time and share one GPU.

Continuous batching at step-chunk granularity:
  * requests wait in an arrival queue (FIFO);
  * a request is admitted when a slot is free and the device footprint of its
    run (columns + workspace, from the library's sizing calls) fits the HBM
    budget next to the runs already resident;
  * every tick advances all resident runs together with amber_step_batch by
    one chunk of steps (a run closer than a chunk to its end advances by what
    it has left), so requests that arrived while others were running overlap
    with them on the device;
  * a run that has finished has its invariants and digest read back (its
    completion time), releases its slot and memory, and queued requests are
    admitted on the next tick;
  * a run alone on the device with no request waiting runs all its remaining
    steps in one amber_step call paced by the host, as a plain run does.

A run's arithmetic never depends on the batch it is in, its slot or its
admission time: its random stream is keyed by (seed, request id) and every
kernel body is the single-run one, so each result equals the run alone.

The plain baseline serves the same stream one request at a time, in arrival
order, with amber_step (one launch per step).
"""
import time
from collections import deque

import numpy as np

from . import amber as A


def _desc_for(req):
    return A.make_desc(req["model"], req["n"], req.get("L", 0), req.get("seed", 0), req["stream"],
                       req.get("wealth_init", 1), tuple(req.get("beta", (1, 20))),
                       tuple(req.get("gamma", (1, 100))), req.get("initial_infected", 0))


def footprint(req):
    """Device bytes the run occupies while resident."""
    return A.footprint_bytes(_desc_for(req))


def _make(req):
    return A.Population(req["model"], req["n"], L=req.get("L", 0), seed=req.get("seed", 0),
                        stream_id=req["stream"], wealth_init=req.get("wealth_init", 1),
                        beta=tuple(req.get("beta", (1, 20))), gamma=tuple(req.get("gamma", (1, 100))),
                        initial_infected=req.get("initial_infected", 0))


class _Run:
    __slots__ = ("req", "pop", "left", "bytes", "admitted")

    def __init__(self, req, pop, nbytes, now):
        self.req, self.pop, self.left, self.bytes, self.admitted = req, pop, req["steps"], nbytes, now


def _summary(records, work, t_start, t_end):
    lat = np.array([r["latency_s"] for r in records]) if records else np.zeros(1)
    return dict(requests=len(records), agent_steps=int(work), seconds=t_end - t_start,
                value=work / max(t_end - t_start, 1e-9),
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                records=records)


def serve(requests, budget_bytes, chunk=50, max_slots=512, time_scale=1.0, torch=None,
          log=None):
    """Serve `requests` (dicts with arrival [s], model, n, steps, stream, ...)
    replayed open-loop against the wall clock (arrival times divided by
    time_scale).  Returns throughput, p50/p99 latency and per-request records
    (digest, latency, admission wait)."""
    reqs = sorted(requests, key=lambda r: r["arrival"])
    for r in reqs:
        r["_bytes"] = footprint(r)
        if r["_bytes"] == 0 or r["_bytes"] > budget_bytes:
            raise ValueError(f"request {r['stream']} cannot fit the HBM budget")
    pending = deque(reqs)          # not yet arrived
    queue = deque()                # arrived, waiting for admission
    resident = []
    used = 0
    records = []
    work = 0
    ticks = 0
    t_start = time.perf_counter()
    now = lambda: (time.perf_counter() - t_start) * time_scale

    while pending or queue or resident:
        clock = now()
        while pending and pending[0]["arrival"] <= clock:
            queue.append(pending.popleft())
        # admission by footprint, FIFO, no overtaking
        while queue and len(resident) < max_slots and used + queue[0]["_bytes"] <= budget_bytes:
            req = queue.popleft()
            resident.append(_Run(req, _make(req), req["_bytes"], now()))
            used += req["_bytes"]
        if not resident:
            if pending:
                wait = (pending[0]["arrival"] - now()) / time_scale
                if wait > 0:
                    time.sleep(min(wait, 0.05))
            continue
        # one tick: every resident run advances by min(chunk, what it has left);
        # a run alone on the device with nothing queued behind it runs all its
        # steps in one call, paced by the host (the early stop and, on big
        # grids, the tiled-then-gather mode take effect as for a plain run)
        if len(resident) == 1 and not queue and not (pending and pending[0]["arrival"] <= now()):
            run = resident[0]
            run.pop.tune(sir_poll=A.POLL_PACED)
            run.pop.step(run.left)
            run.left = 0
            by_len = {}
        else:
            by_len = {}
            for run in resident:
                by_len.setdefault(min(chunk, run.left), []).append(run)
        for k, runs in by_len.items():
            A.step_batch([r.pop for r in runs], k)
            for r in runs:
                r.left -= k
        ticks += 1
        still = []
        for run in resident:
            if run.left == 0:
                inv = run.pop.invariants()          # waits for the run's work
                done = now()
                req = run.req
                records.append(dict(id=req["stream"], model=req["model"], n=req["n"],
                                    steps=req["steps"], digest=inv["digest"], invariants=inv,
                                    latency_s=(done - req["arrival"]) / time_scale,
                                    wait_s=(run.admitted - req["arrival"]) / time_scale))
                work += req["n"] * req["steps"]
                run.pop.release()
                used -= run.bytes
            else:
                still.append(run)
        resident = still
        if log and ticks % 100 == 0:
            log(f"serve: t={now():.1f}s resident={len(resident)} queued={len(queue)} "
                f"done={len(records)} used={used / 2**30:.1f} GiB")
    out = _summary(records, work, t_start, time.perf_counter())
    out["ticks"] = ticks
    return out


def serve_plain(requests, time_scale=1.0, log=None):
    """FIFO, one request at a time, one launch per step."""
    reqs = sorted(requests, key=lambda r: r["arrival"])
    records = []
    work = 0
    t_start = time.perf_counter()
    now = lambda: (time.perf_counter() - t_start) * time_scale
    for i, req in enumerate(reqs):
        wait = (req["arrival"] - now()) / time_scale
        if wait > 0:
            time.sleep(wait)
        start = now()
        pop = _make(req)
        pop.step(req["steps"])
        inv = pop.invariants()
        done = now()
        pop.release()
        records.append(dict(id=req["stream"], model=req["model"], n=req["n"], steps=req["steps"],
                            digest=inv["digest"], invariants=inv,
                            latency_s=(done - req["arrival"]) / time_scale,
                            wait_s=(start - req["arrival"]) / time_scale))
        work += req["n"] * req["steps"]
        if log and i % 200 == 0:
            log(f"serve_plain: {i}/{len(reqs)} t={now():.1f}s")
    return _summary(records, work, t_start, time.perf_counter())


def alone_digest(req):
    """The request's run stepped alone (reference for the mix-equality check)."""
    pop = _make(req)
    pop.step(req["steps"])
    d = pop.invariants()["digest"]
    pop.release()
    return d
