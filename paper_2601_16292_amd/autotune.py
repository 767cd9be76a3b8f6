"""Autotuner: choose launch shapes per (device, model, size, grid, call length).

Every knob of ``amber_set_tuning`` changes only speed, never results: all
arithmetic is integer and every random word is addressed by agent id and step.
The tuner runs each candidate on a representative run of the requested model
and size, times it with HIP events on the run's stream, checks that every
candidate ends with the same digest (a candidate that disagrees is an error,
not a slower choice), and caches the fastest tuning as JSON.

The cache key holds what the library's own automatic choices switch on:
the device, the model, floor(log2 N), the grid bucket floor(log2 L^2), the
call-length class (under 16 steps, 16 to 127, 128 or more) and a hash of the
kernel sources, so an entry measured with other kernels is never reused.

Usage:
    best = autotune.tune(model, n, L=0, steps=50)      # measures (or cache hit)
    autotune.apply(pop, steps=50)                      # sets pop's tuning from the cache
"""
import hashlib
import json
import math
import os
import time

from . import amber as A

DEFAULT_CACHE = os.environ.get("AMBER_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "amber",
                                            "autotune.json"))
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def size_bucket(n):
    """Population-size bucket: floor(log2 n) (runs within a factor 2 share a tuning)."""
    return int(math.floor(math.log2(max(1, n))))


def grid_bucket(L):
    """Grid bucket: floor(log2 L^2) (0 for models without a grid)."""
    return int(math.floor(math.log2(L * L))) if L and L > 1 else 0


def call_class(steps):
    """Call-length class: the library's automatic SIR count mode changes at
    16 and 128 steps per call."""
    return 0 if steps < 16 else (1 if steps < 128 else 2)


_SRC_HASH = None


def source_hash():
    """Hash of the kernel and runtime sources the tuned library is built from."""
    global _SRC_HASH
    if _SRC_HASH is None:
        h = hashlib.sha256()
        for name in sorted(os.listdir(CSRC)):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
        _SRC_HASH = h.hexdigest()[:16]
    return _SRC_HASH


def device_key(torch):
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(props, 'gcnArchName', props.name)}:{props.multi_processor_count}cu"


def candidates(model, n, steps=50, persistent=True):
    """Launch shapes worth trying for a model, size and call length."""
    if model == A.SIR:
        out = [dict(sir_form=A.SIR_AUTO, sir_count=A.COUNT_AUTO, block=b) for b in (256, 512)]
        for count in (A.COUNT_GATHER, A.COUNT_BOX, A.COUNT_EXCHANGE):
            for block in (128, 256, 512):
                out.append(dict(sir_form=A.SIR_PIPELINED, sir_count=count, block=block))
        for tile, blocks in ((32, (256, 512)), (64, (512, 1024))):
            for block in blocks:
                out.append(dict(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_TILED,
                                sir_tile=tile, block=block))
        if steps > 32:
            # calls long enough for the early stop and the tiled-then-gather
            # switch: also with the host pacing the call (sir_poll 2)
            for block in (256, 512):
                out.append(dict(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_GATHER,
                                block=block, sir_poll=A.POLL_PACED))
                out.append(dict(sir_form=A.SIR_AUTO, sir_count=A.COUNT_AUTO, block=block,
                                sir_poll=A.POLL_PACED))
            for tile in (32, 64):
                out.append(dict(sir_form=A.SIR_PIPELINED, sir_count=A.COUNT_TILED_GATHER,
                                sir_tile=tile, block=512, sir_poll=A.POLL_PACED))
        if persistent:
            for g in (2, 4, 8):
                out.append(dict(sir_form=A.SIR_PERSISTENT, max_groups_per_thread=g))
        return out
    if model == A.WEALTH:
        out = [dict(wealth_form=A.WEALTH_ATOMIC, block=b) for b in (128, 256, 512)]
        out.append(dict(wealth_form=A.WEALTH_EXCHANGE))
        return out
    return [dict(block=b) for b in (64, 128, 256, 512, 1024)]


def _grid_side(model, n, L):
    if model == A.WEALTH:
        return 0
    if L:
        return L
    s = math.isqrt(n)
    return s + 1 if n > s * s + s else s


def _key(dev, model, n, L=0, steps=50):
    return (f"{dev}|model={model}|bucket={size_bucket(n)}|grid={grid_bucket(_grid_side(model, n, L))}"
            f"|calls={call_class(steps)}|src={source_hash()}")


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
    """Seconds for one call of `steps` steps after `warmup` steps (warmup 0:
    the run from its initial state), and the final digest.  Returns
    (None, None) when the tuning is not available for this run."""
    pop = A.Population(model, n, L=L, seed=0, stream_id=0, beta=beta, gamma=gamma)
    try:
        pop.tune(**tuning)
        try:
            if warmup:
                pop.step(warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(pop.stream)
            t0 = time.perf_counter()
            pop.step(steps)
            e1.record(pop.stream)
            torch.cuda.synchronize()
        except A.AmberError as e:
            if e.status == A.E_UNSUPPORTED:
                return None, None
            raise
        # the call's wall time when the host paces it (sir_poll 2 blocks
        # inside the call), otherwise the device time of its launches
        secs = max(e0.elapsed_time(e1) / 1e3, time.perf_counter() - t0)
        digest = pop.invariants()["digest"]
        return secs, digest
    finally:
        pop.release()


def tune(model, n, L=0, steps=50, warmup=5, torch=None, cache_path=DEFAULT_CACHE, force=False,
         beta=(1, 20), gamma=(1, 100), log=None, persistent=True, repeats=1):
    """Best tuning for (device, model, size, grid, call length), measured on
    a run of n agents (best of `repeats` timings per candidate).  Raises if
    two candidates disagree on the result."""
    if torch is None:
        import torch
    dev = device_key(torch)
    cache = load_cache(cache_path)
    key = _key(dev, model, n, L, steps)
    if key in cache and not force:
        return cache[key]["tuning"]
    results = []
    ref_digest = None
    for cand in candidates(model, n, steps, persistent):
        best = None
        for _ in range(max(1, repeats)):
            secs, digest = measure(torch, model, n, cand, L, steps, warmup, beta, gamma)
            if secs is None:
                break
            if ref_digest is None:
                ref_digest = digest
            elif digest != ref_digest:
                raise RuntimeError(f"tuning {cand} changed the result ({digest} != {ref_digest})")
            best = secs if best is None else min(best, secs)
        if best is None:
            continue
        results.append((best, cand))
        if log:
            log(f"autotune: model={model} n={n} {cand}: {best * 1e3:.3f} ms")
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    cache[key] = {"tuning": best, "n": n, "L": L, "steps": steps, "warmup": warmup,
                  "measured_at": time.time(),
                  "ms": {json.dumps(c, sort_keys=True): round(s * 1e3, 4) for s, c in results}}
    save_cache(cache, cache_path)
    return best


def lookup(model, n, torch=None, cache_path=DEFAULT_CACHE, L=0, steps=50):
    """Cached tuning for the key of this run and call length (None when not
    tuned yet)."""
    if torch is None:
        import torch
    entry = load_cache(cache_path).get(_key(device_key(torch), model, n, L, steps))
    return entry["tuning"] if entry else None


def apply(pop, torch=None, cache_path=DEFAULT_CACHE, steps=50):
    """Set a Population's tuning from the cache (no-op when not tuned)."""
    t = lookup(pop.model, pop.n, torch, cache_path, L=pop.info().grid_side, steps=steps)
    if t:
        pop.tune(**t)
    return t
