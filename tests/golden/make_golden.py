"""Write the stored expected values of the full-size parity tests.

Every value here comes from the oracle (``oracle/``) run on the seeded
workloads of ``paper_2601_16292_amd.workloads`` -- nothing is taken from the
GPU path.  Outputs (JSON, in this directory):

  configs.json  wealth N=1000 x 100 steps (full column), random walk
                N=1e6 on 1000x1000 x 1000 steps (digest, invariants, a sample
                of agents), grid SIR N=1e6 on 1000x1000 x 500 steps (digest and
                invariants at several steps);
  sweep.json    the 256-replicate SIR sweep, 300 steps: per-replicate digest
                and S/I/R counts (slow: run with --sweep, uses a process pool);
  served_sample.json
                a stratified sample of the 10,000-request served stream: for
                each model, the first request of each N decile (log-spaced
                over [1e4, 1e7]) plus the model's heaviest request (largest
                N x steps); digest and invariants after all its steps
                (--served, process pool);
  sir_2p27.json grid SIR at N = 2^27 (L = round(sqrt N) = 11585), beta 1/20,
                gamma 1/100, key (0, 0), 500 steps: digest and S/I/R at
                checkpoints (--big; about half an hour on one core).

Usage:  python tests/golden/make_golden.py [--sweep | --served | --big] [--jobs N]
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2601_16292_amd import workloads as W  # noqa: E402

WALK_SAMPLE_SEED = 12345
WALK_SAMPLE = 4096


def _inv(run):
    inv = run.invariants()
    inv["digest"] = run.digest()
    inv["step"] = run.t
    return inv


def configs():
    out = {}
    c = W.WEALTH_1K
    r = O.OracleRun(O.WEALTH, c["n"], seed=c["seed"], stream=c["stream"], wealth_init=c["wealth_init"])
    marks = {}
    for t in (1, 10, c["steps"]):
        r.step(t - r.t)
        marks[str(t)] = _inv(r)
    out["wealth_1k"] = dict(config=c, checkpoints=marks, wealth=r.w.tolist())
    print("wealth done", flush=True)

    c = W.WALK_1M
    r = O.OracleRun(O.RANDOM_WALK, c["n"], c["L"], seed=c["seed"], stream=c["stream"])
    marks = {}
    for t in (1, 100, c["steps"]):
        r.step(t - r.t)
        marks[str(t)] = _inv(r)
    ids = np.sort(np.random.default_rng(WALK_SAMPLE_SEED).choice(c["n"], WALK_SAMPLE, replace=False))
    out["walk_1m"] = dict(config=c, checkpoints=marks, sample_ids=ids.tolist(),
                          sample_x=r.x[ids].tolist(), sample_y=r.y[ids].tolist())
    print("walk done", flush=True)

    c = W.SIR_1M
    r = O.OracleRun(O.SIR, c["n"], c["L"], seed=c["seed"], stream=c["stream"], beta=c["beta"],
                    gamma=c["gamma"])
    marks = {"0": _inv(r)}
    for t in (1, 10, 100, c["steps"]):
        r.step(t - r.t)
        marks[str(t)] = _inv(r)
        print("sir", t, marks[str(t)], flush=True)
    out["sir_1m"] = dict(config={k: list(v) if isinstance(v, tuple) else v for k, v in c.items()},
                         checkpoints=marks)
    return out


def _sweep_one(run):
    r = O.OracleRun(O.SIR, run["n"], run["L"], seed=run["seed"], stream=run["stream"],
                    beta=run["beta"], gamma=run["gamma"]).step(run["steps"])
    inv = _inv(r)
    return dict(stream=run["stream"], n=run["n"], beta=list(run["beta"]), **inv)


def sweep(jobs):
    runs = W.sir_sweep()
    order = sorted(range(len(runs)), key=lambda i: -runs[i]["n"])   # big first
    with Pool(jobs) as pool:
        res = pool.map(_sweep_one, [runs[i] for i in order], chunksize=1)
    res.sort(key=lambda d: d["stream"])
    return dict(steps=runs[0]["steps"], runs=res)


SERVED_DECILES = 10


def served_sample():
    """Indices of the stratified sample of the served stream (inputs only)."""
    reqs = W.served_stream()
    edges = np.logspace(4, 7, SERVED_DECILES + 1)
    picked = []
    for m in range(3):
        mine = [r for r in reqs if r["model"] == m]
        for d in range(SERVED_DECILES):
            lo, hi = edges[d], edges[d + 1]
            for r in mine:
                if lo <= r["n"] < hi or (d == SERVED_DECILES - 1 and r["n"] == hi):
                    picked.append(r["id"])
                    break
        heavy = max(mine, key=lambda r: (r["n"] * r["steps"], -r["id"]))
        if heavy["id"] not in picked:
            picked.append(heavy["id"])
    return sorted(picked)


def _served_one(req):
    r = O.OracleRun(req["model"], req["n"], req["L"], seed=req["seed"], stream=req["stream"],
                    wealth_init=req.get("wealth_init", 1), beta=tuple(req.get("beta", (1, 20))),
                    gamma=tuple(req.get("gamma", (1, 100)))).step(req["steps"])
    inv = _inv(r)
    return dict(id=req["id"], model=req["model"], n=req["n"], steps=req["steps"], **inv)


def served(jobs):
    reqs = W.served_stream()
    ids = served_sample()
    todo = sorted((reqs[i] for i in ids), key=lambda r: -r["n"] * r["steps"])
    with Pool(jobs) as pool:
        res = pool.map(_served_one, todo, chunksize=1)
    res.sort(key=lambda d: d["id"])
    return dict(sample="per model: first request of each N decile (log-spaced over [1e4, 1e7]) "
                       "and the heaviest request (largest N x steps)", runs=res)


BIG_CHECKPOINTS = (0, 1, 10, 50, 100, 150, 200, 300, 400, 500)


def big():
    c = W.SIR_BIG
    r = O.OracleRun(O.SIR, c["n"], c["L"], seed=c["seed"], stream=c["stream"], beta=c["beta"],
                    gamma=c["gamma"])
    marks = {}
    for t in BIG_CHECKPOINTS:
        r.step(t - r.t)
        marks[str(t)] = _inv(r)
        print("sir 2^27", t, marks[str(t)], flush=True)
    cfg = {k: list(v) if isinstance(v, tuple) else v for k, v in c.items()}
    cfg["L"] = r.L
    cfg["steps"] = BIG_CHECKPOINTS[-1]
    return dict(config=cfg, checkpoints=marks)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--served", action="store_true")
    ap.add_argument("--big", action="store_true")
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    args = ap.parse_args()
    t0 = time.time()
    if args.sweep:
        data = sweep(args.jobs)
        path = os.path.join(HERE, "sweep.json")
    elif args.served:
        data = served(args.jobs)
        path = os.path.join(HERE, "served_sample.json")
    elif args.big:
        data = big()
        path = os.path.join(HERE, "sir_2p27.json")
    else:
        data = configs()
        path = os.path.join(HERE, "configs.json")
    data["generated_by"] = "tests/golden/make_golden.py (oracle only)"
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote", path, f"in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
