"""Autotuner: choose launch shapes per (device, model, population-size bucket).

Every knob of ``amber_set_tuning`` changes only speed, never results: all
arithmetic is integer and every random word is addressed by agent id and step.
The tuner runs each candidate on a representative run of the requested model
and size, times a window of steps with HIP events on the run's stream, checks
that every candidate ends with the same digest (a candidate that disagrees is
an error, not a slower choice), and caches the fastest tuning as JSON.

Usage:
    best = autotune.tune(model, n, L=0, steps=50)      # measures (or cache hit)
    autotune.apply(pop)                                # sets pop's tuning from the cache
"""
import json
import math
import os
import time

from . import amber as A

DEFAULT_CACHE = os.environ.get("AMBER_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "amber",
                                            "autotune.json"))


def size_bucket(n):
    """Population-size bucket: floor(log2 n) (runs within a factor 2 share a tuning)."""
    return int(math.floor(math.log2(max(1, n))))


def device_key(torch):
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(props, 'gcnArchName', props.name)}:{props.multi_processor_count}cu"


def candidates(model, n):
    """Launch shapes worth trying for a model and size."""
    if model == A.SIR:
        out = []
        for count in (A.COUNT_GATHER, A.COUNT_BOX, A.COUNT_EXCHANGE):
            for block in (128, 256, 512):
                out.append(dict(sir_form=A.SIR_PIPELINED, sir_count=count, block=block))
        for tile, blocks in ((32, (256, 512)), (64, (512, 1024))):
            for block in blocks:
                out.append(dict(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_TILED,
                                sir_tile=tile, block=block))
        for g in (2, 4, 8):
            out.append(dict(sir_form=A.SIR_PERSISTENT, max_groups_per_thread=g))
        return out
    if model == A.WEALTH:
        out = [dict(wealth_form=A.WEALTH_ATOMIC, block=b) for b in (128, 256, 512)]
        out.append(dict(wealth_form=A.WEALTH_EXCHANGE))
        return out
    return [dict(block=b) for b in (64, 128, 256, 512, 1024)]


def _key(dev, model, n):
    return f"{dev}|model={model}|bucket={size_bucket(n)}"


def load_cache(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def measure(torch, model, n, tuning, L=0, steps=50, warmup=5, beta=(1, 20), gamma=(1, 100)):
    """Seconds for `steps` steps after `warmup` steps, and the final digest.
    Returns (None, None) when the tuning is not available for this run."""
    pop = A.Population(model, n, L=L, seed=0, stream_id=0, beta=beta, gamma=gamma)
    try:
        pop.tune(**tuning)
        try:
            pop.step(warmup)
        except A.AmberError as e:
            if e.status == A.E_UNSUPPORTED:
                return None, None
            raise
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(pop.stream)
        pop.step(steps)
        e1.record(pop.stream)
        torch.cuda.synchronize()
        secs = e0.elapsed_time(e1) / 1e3
        digest = pop.invariants()["digest"]
        return secs, digest
    finally:
        pop.release()


def tune(model, n, L=0, steps=50, warmup=5, torch=None, cache_path=DEFAULT_CACHE, force=False,
         beta=(1, 20), gamma=(1, 100), log=None):
    """Best tuning for (device, model, size bucket), measured on a run of n
    agents.  Raises if two candidates disagree on the result."""
    if torch is None:
        import torch
    dev = device_key(torch)
    cache = load_cache(cache_path)
    key = _key(dev, model, n)
    if key in cache and not force:
        return cache[key]["tuning"]
    results = []
    ref_digest = None
    for cand in candidates(model, n):
        secs, digest = measure(torch, model, n, cand, L, steps, warmup, beta, gamma)
        if secs is None:
            continue
        if ref_digest is None:
            ref_digest = digest
        elif digest != ref_digest:
            raise RuntimeError(f"tuning {cand} changed the result ({digest} != {ref_digest})")
        results.append((secs, cand))
        if log:
            log(f"autotune: model={model} n={n} {cand}: {secs * 1e3:.3f} ms")
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    cache[key] = {"tuning": best, "n": n, "steps": steps, "measured_at": time.time(),
                  "ms": {json.dumps(c, sort_keys=True): round(s * 1e3, 4) for s, c in results}}
    save_cache(cache, cache_path)
    return best


def lookup(model, n, torch=None, cache_path=DEFAULT_CACHE):
    """Cached tuning for the bucket of n (None when not tuned yet)."""
    if torch is None:
        import torch
    entry = load_cache(cache_path).get(_key(device_key(torch), model, n))
    return entry["tuning"] if entry else None


def apply(pop, torch=None, cache_path=DEFAULT_CACHE):
    """Set a Population's tuning from the cache (no-op when not tuned)."""
    t = lookup(pop.model, pop.n, torch, cache_path)
    if t:
        pop.tune(**t)
    return t
