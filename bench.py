"""Benchmark of the columnar ABM hot path on one MI355X.

Headline workload (the metric's case): grid SIR with N = 1e6 agents on a
1000 x 1000 torus, beta = 1/20, gamma = 1/100, 0.1% initially infected,
key (0, 0), 500 steps.  One bench step = one whole run of that workload:
amber_init_population on device buffers already allocated in HBM, one
500-step amber_step call (move, cell binning, neighbour counts, transitions
for every agent and step) and amber_invariants (the run's S/I/R counts and
digest on the host).  W untimed runs, then K timed runs (defaults W = 5,
K = 20); value = N * 500 * K / wall time of the K runs.

Prints ONE JSON line: agent-steps/s of the headline, the roofline of its
dominant kernel (algorithmic bytes per launch / average launch time from HIP
events on the library's stream, measured traffic from the committed counter
summary), the CPU oracle timed on a bounded sample, and extra blocks: the
wealth and random-walk models at 1e3 / 1e6 agents, the per-step kernels and
whole runs at N = 2^27 (out of cache), the 256-replicate sweep (plain against
batched), a served stream subset (continuous batching against a FIFO queue).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
                  [--no-big] [--no-sweep] [--serve N] [--headline-only]
                  [--tuning JSON | --cached-tuning] [--counter-run]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, vendor figure
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2601_16292_amd", "csrc", f)
                  for f in ("amber_device.hip", "amber_device_common.h", "amber_tiled.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
BIG_GOLDEN = os.path.join(ROOT, "tests", "golden", "sir_2p27.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# ------------------------------------------------------------------ algorithmic bytes

def sir_step_bytes(n, L, infected, susceptible=1):
    """Algorithmic bytes of one SIR step with `infected` agents infected at its
    start: positions read and written (16 B/agent), state read and written
    (2 B/agent), the L*L count grid cleared once and read once (8 B/cell) and
    one 8-B read-modify-write per infected agent.  With no susceptible agent
    left no count is read, and the step needs only the columns."""
    return 18 * n + ((8 * L * L + 8 * infected) if susceptible else 0)


def sir_gather_body_bytes(n, L, counts, calls):
    """Algorithmic bytes of the gather-mode body launches (call-relative steps
    1 .. len-1 of each call).  counts[k] = (S, I) at the start of step k of
    the region.  Launch j is the first of its call with S = 0 three steps
    back; it runs every remaining step of the call in registers (one pass
    over the columns, 18 B/agent), and the later launches of the call move
    nothing."""
    total, a = 0, 0
    for ln in calls:
        for j in range(1, ln):
            if j >= 3 and counts[a + j - 3][0] == 0:
                total += 18 * n
                break
            s, i = counts[a + j]
            total += sir_step_bytes(n, L, i, s)
        a += ln
    return total


def tile_step_bytes(n, L):
    """Bytes one step of the tiled SIR mode must move in its own layout: each
    agent's 8-byte record read and written, and the L*L count grid written
    and read once."""
    return 16 * n + 8 * L * L


def wealth_step_bytes(n, donors):
    """Wealth read and written (8 B per agent) plus one 8-B RMW per donor."""
    return 8 * n + 8 * donors


def price_sir_run(n, L, counts, times, steps):
    """Algorithmic bytes of every priced kernel of one SIR call of `steps`
    steps from counts[0] (S, I at the start of each step).  The tiled bodies
    of a tiled (then gather) call are priced with the method's bytes per step
    (18 N + 8 L^2 + 8 I_t), their record bytes kept beside them; a gather
    segment after them starts where the tiled part ended."""
    priced, extra = {}, {}
    tiled = times.get("sir_tile_body", (0, 0))[0]
    start = 0
    if tiled:
        k = tiled + 1                    # head (step 0), bodies 1..k-1
        if "sir_body" not in times and "sir_head" not in times:
            k = steps                    # the call stayed tiled
        priced["sir_tile_body"] = sum(sir_step_bytes(n, L, counts[t][1], counts[t][0])
                                      for t in range(1, tiled + 1))
        extra["sir_tile_body"] = {"record_bytes_per_launch": tile_step_bytes(n, L)}
        start = k
    if "sir_body" in times:
        priced["sir_body"] = sir_gather_body_bytes(n, L, counts[start:], [steps - start])
    if "sir_head" in times:
        s0, i0 = counts[start]
        priced["sir_head"] = sir_step_bytes(n, L, i0, s0)
    if "sir_persistent" in times:
        priced["sir_persistent"] = sum(sir_step_bytes(n, L, i, s) for s, i in counts[:steps])
    return priced, extra


def roofline_for(times, bytes_per_kernel_total, traffic, extra=None):
    """Dominant kernel = largest total device time among those we can price."""
    best = None
    for name, (launches, total_ms) in times.items():
        if name not in bytes_per_kernel_total or launches == 0:
            continue
        if best is None or total_ms > best[2]:
            best = (name, launches, total_ms)
    if best is None:
        return None
    name, launches, total_ms = best
    avg_s = total_ms / launches / 1e3
    bytes_per_launch = bytes_per_kernel_total[name] / launches
    achieved = bytes_per_launch / avg_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "kernel": name,
           "launches": launches, "avg_launch_us": round(avg_s * 1e6, 3),
           "algorithmic_bytes_per_launch": int(bytes_per_launch)}
    if extra and name in extra:
        out.update(extra[name])
    if traffic and name in traffic:
        # the number of launches of a call can vary (the host stops enqueueing
        # once one launch has run the call's remaining steps): bytes of the
        # whole call over this run's launches
        out["traffic"] = int(traffic[name]["bytes_per_call"] / launches)
        out["traffic_launches_in_counter_run"] = traffic[name]["launches_per_call"]
    return out


def load_traffic(tuning):
    """HBM traffic per kernel of one headline call under `tuning`, from the
    committed rocprofv3 counter summary: {kernel: entry}, empty when no entry
    was taken with this tuning or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("source_sha") != kernel_source_sha():
        return {}
    return {e["kernel"]: e for e in t.get("entries", []) if e.get("tuning") == tuning}


# ------------------------------------------------------------------ timing helpers

def timed_steps(torch, pop, steps, chunk):
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(pop.stream)
    done = 0
    while done < steps:
        c = min(chunk or steps, steps - done)
        pop.step(c)
        done += c
    ev1.record(pop.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return max(wall, ev0.elapsed_time(ev1) / 1e3)


class SirRuns:
    """Whole runs of one SIR workload on device buffers allocated once."""

    def __init__(self, A, c, tuning):
        self.A, self.c, self.tuning = A, c, tuning or {}
        first = A.Population(A.SIR, c["n"], L=c["L"], seed=c["seed"], stream_id=c["stream"],
                             beta=c["beta"], gamma=c["gamma"])
        self.bufs = dict(first.cols, workspace=first.workspace)
        self.L = first.info().grid_side
        first.release()

    def make(self):
        A, c = self.A, self.c
        p = A.Population(A.SIR, c["n"], L=c["L"], seed=c["seed"], stream_id=c["stream"],
                         beta=c["beta"], gamma=c["gamma"], buffers=self.bufs)
        if self.tuning:
            p.tune(**self.tuning)
        return p

    def run(self, profile=False):
        """init + one call of every step + invariants (host); returns the
        invariants (and the per-kernel times when profiling)."""
        p = self.make()
        if profile:
            p.profile(True)
        p.step(self.c["steps"])
        times = p.kernel_times() if profile else None
        inv = p.invariants()
        p.release()
        return inv, times

    def counts(self):
        """(S, I) at the start of every step of the run."""
        p = self.make()
        out = []
        for _ in range(self.c["steps"]):
            v = p.invariants()
            out.append((v["n_s"], v["n_i"]))
            p.step(1)
        p.release()
        return out


def headline(torch, A, W, K, tuning):
    from paper_2601_16292_amd import workloads as WL
    c = WL.SIR_1M
    runs = SirRuns(A, c, tuning)
    for _ in range(W):
        runs.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    digests = set()
    inv = None
    for _ in range(K):
        inv, _ = runs.run()
        digests.add(inv["digest"])
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    # instrumented replay of one run: per-kernel launch times
    _, times = runs.run(profile=True)
    counts = runs.counts()
    return dict(secs=secs, inv=inv, same=len(digests) == 1, times=times, counts=counts,
                n=c["n"], L=runs.L, steps=c["steps"], bufs=runs)


# ------------------------------------------------------------------ extras

def wealth_bench(torch, A, n, W, K, chunk=0, form=0):
    pop = A.Population(A.WEALTH, n, seed=0, stream_id=0, wealth_init=1)
    pop.tune(wealth_form=form)
    pop.step(W)
    secs = timed_steps(torch, pop, K, chunk)
    inv = pop.invariants()
    pop.release()
    return secs, inv


def walk_bench(torch, A, n, L, K):
    pop = A.Population(A.RANDOM_WALK, n, L=L, seed=0, stream_id=0)
    secs = timed_steps(torch, pop, K, 0)
    inv = pop.invariants()
    pop.release()
    return secs, inv


def extras(torch, A):
    out = {}
    s, winv = wealth_bench(torch, A, 1000, 0, 100)
    out["wealth_1k"] = {"value": round(1000 * 100 / s, 1), "unit": "agent-steps/s",
                        "steps": 100, "ms_total": round(s * 1e3, 4),
                        "wealth_sum": winv["wealth_sum"], "digest": winv["digest"]}
    for form, label in ((0, "wealth_1m"), (1, "wealth_1m_atomic")):
        s, winv = wealth_bench(torch, A, 1_000_000, 10, 200, form=form)
        out[label] = {"value": round(1e6 * 200 / s, 1), "unit": "agent-steps/s",
                      "steps": 200, "ms_per_step": round(s * 1e3 / 200, 5),
                      "wealth_sum": winv["wealth_sum"]}
    s, rinv = walk_bench(torch, A, 1_000_000, 1000, 1000)
    out["walk_1m"] = {"value": round(1e6 * 1000 / s, 1), "unit": "agent-steps/s",
                      "steps": 1000, "ms_total": round(s * 1e3, 4),
                      "out_of_bounds": rinv["out_of_bounds"], "digest": rinv["digest"]}
    return out


def roofline_big(torch, A, log2n):
    """Per-step kernels at an out-of-cache size (columns far above the 256 MB
    last-level cache): average launch time from HIP events on the library's
    stream, algorithmic bytes per launch, achieved GB/s against HBM peak;
    then whole 500-step SIR runs in several modes."""
    n = 1 << log2n
    res = {"n_agents": n}

    def priced(name, times, bytes_per_launch):
        launches, total_ms = times[name]
        avg = total_ms / launches / 1e3
        gbs = bytes_per_launch / avg / 1e9
        return {"kernel": name, "launches": launches, "avg_launch_us": round(avg * 1e6, 2),
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "achieved_GBs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / PEAK_HBM_GBS, 4)}

    # random walk, one step per launch (16 B per agent-step)
    pop = A.Population(A.RANDOM_WALK, n, L=1000)
    pop.step(1)
    pop.profile(True)
    for _ in range(8):
        pop.step(1)
    res["walk_step"] = priced("walk", pop.kernel_times(), 16 * n)
    pop.release()
    torch.cuda.empty_cache()

    # wealth: partition exchange and the global atomic scatter at n, and the
    # exchange at 2^24; 8 B per agent + 8 B per donor
    for nx, form, name, label in (((1 << 24), 2, "wealth_exchange", "wealth_exchange_2p24"),
                                  (n, 2, "wealth_exchange", "wealth_exchange"),
                                  (n, 1, "wealth_step", "wealth_step")):
        pop = A.Population(A.WEALTH, nx, wealth_init=1)
        pop.tune(wealth_form=form)
        pop.step(2)
        (w,) = pop.read()
        donors = int((w > 0).sum())
        del w
        pop.profile(True)
        pop.step(3)
        res[label] = priced(name, pop.kernel_times(), wealth_step_bytes(nx, donors))
        res[label]["donors_after_step_2"] = donors
        pop.release()
        torch.cuda.empty_cache()

    # SIR per-step bodies at step 31, priced with the method's bytes
    # 18 N + 8 L^2 + 8 I_t; the box mode's grid bytes are booked on its
    # stencil kernel, the tiled mode's own record bytes are shown beside
    for label, tu, kernel in (("gather", dict(sir_form=1, sir_count=1), "sir_body"),
                              ("box", dict(sir_form=1, sir_count=2), "sir_body_box"),
                              ("tiled32", dict(sir_form=1, sir_count=4, sir_tile=32), "sir_tile_body"),
                              ("tiled64", dict(sir_form=1, sir_count=4, sir_tile=64), "sir_tile_body")):
        pop = A.Population(A.SIR, n, L=0, beta=(1, 20), gamma=(1, 100))
        L = pop.info().grid_side
        pop.tune(**tu)
        pop.step(30)
        i_t = pop.invariants()["n_i"]
        pop.profile(True)
        pop.step(2)        # the body is step 31
        times = pop.kernel_times()
        step_bytes = 18 * n + 8 * L * L + 8 * i_t
        if label == "box":
            entry = priced(kernel, times, step_bytes - 8 * L * L)
            entry["box_kernel"] = priced("sir_box", times, 8 * L * L)
            both = (times[kernel][1] / times[kernel][0] + times["sir_box"][1] / times["sir_box"][0]) / 1e3
            entry["step_GBs"] = round(step_bytes / both / 1e9, 1)
            entry["step_frac_of_hbm_peak"] = round(step_bytes / both / 1e9 / PEAK_HBM_GBS, 4)
        else:
            entry = priced(kernel, times, step_bytes)
        if label.startswith("tiled"):
            avg = times[kernel][1] / times[kernel][0] / 1e3
            rb = tile_step_bytes(n, L)
            entry["record_bytes_per_launch"] = rb
            entry["record_frac_of_hbm_peak"] = round(rb / avg / 1e9 / PEAK_HBM_GBS, 4)
            entry["call_kernels_us"] = {k: round(v[1] / max(1, v[0]) * 1e3, 1) for k, v in times.items()}
        entry.update({"grid_side": L, "infected": i_t})
        res[f"sir_body_{label}"] = entry
        pop.release()
        torch.cuda.empty_cache()

    # view primitives on 2^27-row columns: a full and a filtered int32
    # update (8 B per row, plus 4 B per row of predicate), a float32 update,
    # and int32 / float32 scatter-adds of 2^25 entries (ids and values read,
    # one 8-B read-modify-write per entry)
    res["views"] = view_roofline(torch, A, n)
    torch.cuda.empty_cache()

    # whole SIR runs at this size: 499 steps in one call after one step,
    # in the automatic mode (the gather mode when the call is not paced;
    # tiled, then gather when it is), all gather and all tiled
    runs = {}
    for label, tu in (("auto", {}), ("auto_paced", dict(sir_poll=2)),
                      ("gather", dict(sir_form=1, sir_count=1)),
                      ("tiled32", dict(sir_form=1, sir_count=4, sir_tile=32))):
        pop = A.Population(A.SIR, n, L=0, beta=(1, 20), gamma=(1, 100))
        if tu:
            pop.tune(**tu)
        pop.step(1)
        secs = timed_steps(torch, pop, 499, 0)
        inv = pop.invariants()
        runs[label] = {"seconds": round(secs, 4), "agent_steps_per_s": round(n * 499 / secs, 1),
                       "digest": inv["digest"], "n_s": inv["n_s"], "n_i": inv["n_i"],
                       "n_r": inv["n_r"]}
        pop.release()
        torch.cuda.empty_cache()
    digests = {v["digest"] for v in runs.values()}
    runs["identical_outputs"] = len(digests) == 1
    try:
        with open(BIG_GOLDEN) as f:
            gold = json.load(f)
        if gold["config"]["n"] == n:
            runs["oracle_digest_at_500"] = gold["checkpoints"]["500"]["digest"]
            runs["matches_oracle"] = digests == {gold["checkpoints"]["500"]["digest"]}
    except (OSError, ValueError, KeyError):
        pass
    res["sir_whole_run_500_steps"] = runs
    return res


# The paper's Table 1 (AMBER vectorized, Apple Silicon laptop, ms per 50-step
# run): context only, another machine and its own model variants.
PAPER_TABLE1_MS = {"wealth": {500: 4.4, 1000: 6.4, 5000: 21.0},
                   "random_walk": {500: 2.7, 1000: 2.7, 5000: 6.2},
                   "sir": {500: 95.0, 1000: 119.0, 5000: 687.0}}


def paper_models(torch, A, sizes=(500, 1000, 5000), steps=50, reps=20):
    """The paper's benchmark models at its own sizes (Sec. 5.1.2, 50 steps):
    wealth transfer, the continuous clamped walk (100 x 100) and the
    continuous SIR (radius 5, p = 0.1, recovery after 14 days, five
    infected).  One run = init, 50 steps, result on the host; median of
    `reps` runs."""
    import statistics
    out = {}

    def run_wealth(n):
        p = A.Population(A.WEALTH, n, wealth_init=1)
        p.step(steps)
        p.invariants()
        p.release()

    def run_cont(n, sir):
        g = A.ContRun(n, sir=sir)
        g.step(steps)
        g.stream.synchronize()

    for name, fn in (("wealth", run_wealth), ("random_walk", lambda n: run_cont(n, False)),
                     ("sir", lambda n: run_cont(n, True))):
        out[name] = {}
        for n in sizes:
            fn(n)
            times = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn(n)
                times.append(time.perf_counter() - t0)
            ms = statistics.median(times) * 1e3
            out[name][str(n)] = {"ms_per_run": round(ms, 4),
                                 "agent_steps_per_s": round(n * steps / ms * 1e3, 1),
                                 "paper_amber_ms": PAPER_TABLE1_MS[name][n]}
    out["note"] = ("median wall time of a whole run (init, 50 steps, result on the host) on one "
                   "MI355X; paper_amber_ms is the paper's Table 1 AMBER (vectorized) figure on an "
                   "Apple Silicon laptop, context only; the wealth rule lets a donor draw itself "
                   "(the paper's listing), the walk and SIR are the continuous-space models")
    return out


def view_roofline(torch, A, n, m=1 << 25):
    out = {"rows": n, "scatter_entries": m}
    g = torch.Generator(device="cuda").manual_seed(7)
    col = torch.randint(-1000, 1000, (n,), dtype=torch.int32, device="cuda", generator=g)
    colf = torch.rand(n, dtype=torch.float32, device="cuda", generator=g)
    pred = torch.randint(-5, 6, (n,), dtype=torch.int32, device="cuda", generator=g)
    ids = torch.randint(0, n, (m,), dtype=torch.int32, device="cuda", generator=g)
    vals = torch.randint(-9, 9, (m,), dtype=torch.int32, device="cuda", generator=g)
    valsf = torch.rand(m, dtype=torch.float32, device="cuda", generator=g)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    def entry(secs, nbytes):
        gbs = nbytes / secs / 1e9
        return {"avg_call_us": round(secs * 1e6, 2), "algorithmic_bytes": int(nbytes),
                "achieved_GBs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / PEAK_HBM_GBS, 4)}

    out["update_full_i32"] = entry(timed(lambda: A.view_update(col, 3, 1)), 8 * n)
    out["update_filtered_i32"] = entry(timed(lambda: A.view_update(col, 1, -1, pred=pred, cmp=">",
                                                                   thr=0)), 12 * n)
    out["update_full_f32"] = entry(timed(lambda: A.view_update(colf, 1.5, 0.25)), 8 * n)
    out["scatter_add_i32"] = entry(timed(lambda: A.scatter_add(col, ids, vals)), 16 * m)
    ws = torch.empty(A.amber_view_scatter_workspace_bytes(A.DT_F32, n, m), dtype=torch.uint8,
                     device="cuda")
    out["scatter_add_f32"] = entry(timed(lambda: A.scatter_add(colf, ids, valsf, workspace=ws),
                                         reps=2), 16 * m)
    out["scatter_add_f32"]["note"] = ("list order: a stable radix sort of the 2^25 (id, position) "
                                      "pairs (7 passes of 4 bits at 2^27 rows), then one pass "
                                      "over the sorted entries")
    return out


def sweep_block(torch, A):
    from paper_2601_16292_amd import sweep as SW, workloads as WL
    runs = WL.sir_sweep()
    log(f"bench: sweep of {len(runs)} SIR replicates, sum N = {sum(r['n'] for r in runs)}")
    forms = {"plain": SW.run_plain(runs, torch), "batched": SW.run_batched(runs, torch),
             "batched_graph": SW.run_batched(runs, torch, graph=True)}
    same = forms["plain"]["digests"] == forms["batched"]["digests"] == forms["batched_graph"]["digests"]
    out = {}
    for k, v in forms.items():
        out[k] = {"value": round(v["value"], 1), "unit": "agent-steps/s",
                  "seconds": round(v["seconds"], 4), "p50_s": round(v["p50_s"], 4),
                  "p99_s": round(v["p99_s"], 4)}
        for extra in ("setup_s", "capture_s", "order"):
            if extra in v:
                out[k][extra] = v[extra] if isinstance(v[extra], str) else round(v[extra], 4)
    out["identical_outputs"] = bool(same)
    out["workload"] = ("256 SIR replicates, N log-uniform in [1e3, 1e6], grid side round(sqrt N), "
                       "beta 16 values 0.01..0.2, gamma 1/100, 300 steps, key (0, r); latency "
                       "from sweep submission to the replicate's invariants on the host")
    return out


def serve_block(torch, A, n_req, scale, budget_gib, chunk):
    from paper_2601_16292_amd import serve as SV, workloads as WL
    reqs = WL.served_stream()[:n_req]
    log(f"bench: served stream of {len(reqs)} requests, time scale {scale}")
    served = SV.serve([dict(r) for r in reqs], budget_bytes=int(budget_gib * 2**30),
                      chunk=chunk, time_scale=scale, log=log)
    plain = SV.serve_plain([dict(r) for r in reqs], time_scale=scale, log=log)
    keys = ("requests", "agent_steps", "seconds", "p50_s", "p99_s")
    entry = {"served": {k: served[k] for k in keys + ("ticks",)},
             "plain": {k: plain[k] for k in keys}}
    entry["served"]["value"] = round(served["value"], 1)
    entry["plain"]["value"] = round(plain["value"], 1)
    da = {r["id"]: r["digest"] for r in served["records"]}
    db = {r["id"]: r["digest"] for r in plain["records"]}
    entry["identical_outputs"] = da == db
    entry.update({"time_scale": scale, "budget_gib": budget_gib, "chunk": chunk,
                  "workload": f"the first {len(reqs)} requests of the 10,000-request stream: "
                              "Poisson arrivals at 50/s (times divided by time_scale), model "
                              "uniform over wealth / random walk / SIR, N log-uniform in "
                              "[1e4, 1e7], steps uniform in [100, 1000]; latency = completion "
                              "(invariants on the host) - arrival"})
    return entry


# ------------------------------------------------------------------ CPU baseline

def _paper_protocol(fn, runs=3):
    """The paper's timing protocol: run three times, drop the slowest sample,
    average the other two; every sample is returned."""
    samples = [fn() for _ in range(runs)]
    kept = sorted(samples)[:-1] if len(samples) > 1 else samples
    return sum(kept) / len(kept), samples


def cpu_baseline(sample_steps, sweep_steps):
    """The oracle (single-threaded C) timed on the host: the headline SIR
    workload's steps 0..sample_steps-1 on one core; the 256-replicate sweep's
    steps 0..sweep_steps-1 with one thread per replicate over the host's
    cores; and the served stream's CPU time extrapolated from per-model rates."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_2601_16292_amd import workloads as WL
    c = WL.SIR_1M

    def sir_sample(steps):
        r = O.OracleRun(O.SIR, c["n"], c["L"], seed=c["seed"], stream=c["stream"],
                        beta=c["beta"], gamma=c["gamma"])
        t0 = time.perf_counter()
        r.step(steps)
        return time.perf_counter() - t0

    sir_sample(10)                                   # warm-up
    avg, samples = _paper_protocol(lambda: sir_sample(sample_steps))
    out = {"value": round(c["n"] * sample_steps / avg, 1), "unit": "agent-steps/s", "cores": 1,
           "kind": "oracle",
           "sample": (f"grid SIR N=1e6 L=1000 beta=1/20 gamma=1/100 key (0,0), steps "
                      f"0..{sample_steps - 1} of the 500-step run from init; single-threaded C "
                      f"oracle (-O2); warm-up, then 3 runs, slowest dropped, other two averaged"),
           "samples_s": [round(x, 4) for x in samples], "host_cpus": os.cpu_count()}

    # config 4: one thread per replicate over all host cores (the oracle's C
    # calls release the GIL), 256 replicates, steps 0..sweep_steps-1; the
    # runs are created (initial state, threshold tables) before the clock
    runs = WL.sir_sweep()
    cores = min(16, os.cpu_count() or 1)

    def sweep_pass(steps):
        order = sorted(runs, key=lambda r: -r["n"])
        made = [O.OracleRun(O.SIR, r["n"], r["L"], seed=r["seed"], stream=r["stream"],
                            beta=r["beta"], gamma=r["gamma"]) for r in order]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda o: o.step(steps), made))
        return time.perf_counter() - t0, sum(r["n"] for r in runs) * steps

    sweep_pass(2)
    work = sum(r["n"] for r in runs) * sweep_steps
    avg_s, s_samples = _paper_protocol(lambda: sweep_pass(sweep_steps)[0])
    out["sweep_all_cores"] = {"value": round(work / avg_s, 1), "unit": "agent-steps/s",
                              "cores": cores, "kind": "oracle",
                              "sample": (f"the 256 sweep replicates, steps 0..{sweep_steps - 1} "
                                         f"of 300, one thread per replicate; 3 runs, slowest "
                                         f"dropped"),
                              "samples_s": [round(x, 4) for x in s_samples]}

    # config 5: per-model oracle rates on a bounded run, extrapolated over the
    # whole 10,000-request stream
    rates = {}
    for model, name in ((O.WEALTH, "wealth"), (O.RANDOM_WALK, "walk"), (O.SIR, "sir")):
        o = O.OracleRun(model, 1_000_000, 1000, seed=0, stream=0)
        t0 = time.perf_counter()
        o.step(10)
        rates[name] = 1e7 / (time.perf_counter() - t0)
    stream = WL.served_stream()
    per = {"wealth": 0, "walk": 0, "sir": 0}
    for q in stream:
        per[("wealth", "walk", "sir")[q["model"]]] += q["n"] * q["steps"]
    secs = sum(per[k] / rates[k] for k in per)
    out["served_stream_extrapolated"] = {
        "cpu_seconds_1_core": round(secs, 1), "agent_steps": sum(per.values()),
        "rates_per_model": {k: round(v, 1) for k, v in rates.items()},
        "kind": "oracle, extrapolation",
        "sample": "each model at N=1e6 (L=1000) for steps 0..9 on one core; the stream's "
                  "agent-steps per model divided by that model's rate"}
    return out


def copy_probe():
    """A plain device copy of exactly 1 GiB, 5 times: the reference for scaling
    rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": a.numel() * 4, "copies": 5}), flush=True)


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed whole runs")
    ap.add_argument("--warmup", type=int, default=5, help="untimed whole runs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-big", action="store_true", help="skip the N = 2^27 measurements")
    ap.add_argument("--big-log2", type=int, default=27)
    ap.add_argument("--no-sweep", action="store_true", help="skip the 256-replicate sweep")
    ap.add_argument("--serve", type=int, default=300,
                    help="serve the first N requests of the 10,000-request stream (0 = skip)")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="arrival clock speed-up (1 = Poisson 50/s in real time)")
    ap.add_argument("--serve-budget-gib", type=float, default=200.0)
    ap.add_argument("--serve-chunk", type=int, default=50)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline (no extras, 2^27, sweep, serve or CPU legs)")
    ap.add_argument("--tuning", default=None, help="JSON tuning for the headline (no autotune)")
    ap.add_argument("--cached-tuning", action="store_true",
                    help="headline tuning from the autotune cache (measure if absent)")
    ap.add_argument("--counter-run", action="store_true",
                    help="only one whole headline run (for rocprofv3 counter passes)")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--cpu-sweep-steps", type=int, default=20)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.copy_probe:
        copy_probe()
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(runs and replicates are independent; see the sharding design notes). "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        sys.exit("bad --steps/--warmup")
    if args.headline_only:
        args.no_extra = args.no_big = args.no_sweep = args.no_cpu = True
        args.serve = 0

    import torch
    from paper_2601_16292_amd import amber as A
    from paper_2601_16292_amd import autotune as AT
    from paper_2601_16292_amd import workloads as WL
    A.lib()
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    torch.cuda.set_device(0)

    c = WL.SIR_1M
    n, L, T = c["n"], c["L"], c["steps"]
    if args.tuning:
        tuning = json.loads(args.tuning)
    else:
        tune = lambda force: AT.tune(A.SIR, n, L=L, steps=T, warmup=0, torch=torch, force=force,
                                     beta=c["beta"], gamma=c["gamma"], log=log,
                                     persistent=False, repeats=2)
        tuning = tune(force=not args.cached_tuning)
    log(f"bench: SIR N={n} L={L} {T} steps per run, warmup={args.warmup} runs, "
        f"timed={args.steps} runs, tuning {tuning}")

    if args.counter_run:
        runs = SirRuns(A, c, tuning)
        inv, _ = runs.run()
        print(json.dumps({"counter_run": True, "tuning": tuning, "digest": inv["digest"]}),
              flush=True)
        return

    h = headline(torch, A, args.warmup, args.steps, tuning)
    secs, inv, times, counts = h["secs"], h["inv"], h["times"], h["counts"]
    work = n * T * args.steps
    value = work / secs
    log(f"bench: {value:.4g} agent-steps/s, {secs * 1e3 / args.steps:.3f} ms per run, "
        f"kernels {times}")

    priced, pextra = price_sir_run(n, L, counts, times, T)
    roof = roofline_for(times, priced, load_traffic(tuning), pextra)
    if roof is not None:
        run_bytes = sum(sir_step_bytes(n, L, i, s) for s, i in counts)
        roof["run_algorithmic_GBs"] = round(run_bytes * args.steps / secs / 1e9, 1)
        roof["pricing"] = ("per step 18 N + 8 L^2 + 8 I_t (positions and state read and written, "
                           "count grid cleared and read, one RMW per infected agent); a step "
                           "with no susceptible agent reads no count (18 N); the gather-mode "
                           "launch that runs a call's remaining steps in registers is one 18 N "
                           "pass, later launches 0")
        if roof["kernel"] == "sir_body":
            roof["limits"] = ("by phase: global atomics while every infected agent is binned; "
                              "dependent byte loads with demand-driven binning; Philox VALU "
                              "work in the launch that finishes the call")
        roof["residency"] = ("the 1e6 working set (about 27 MB) stays in the 256 MB last-level "
                             "cache across steps: a cache-resident fraction, not an HBM one "
                             "(out-of-cache figures under roofline_big)")
    kernels = {k: {"launches": v[0], "avg_us": round(v[1] / max(1, v[0]) * 1e3, 3)}
               for k, v in times.items()}

    out = {
        "metric": "agent-steps/sec (1e6-agent SIR, wealth); sweep p50/p99 latency, batched vs plain",
        "value": round(value, 1),
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded Philox initial state; no dataset)",
        "config": {"workload": "grid SIR, N=1e6 on a 1000x1000 torus, beta=1/20, gamma=1/100, "
                               "0.1% initially infected, key (0,0), 500 steps; one bench step = "
                               "one whole run (init, 500 steps in one call, invariants on the host)",
                   "n_agents": n, "grid_side": L, "steps_per_run": T,
                   "agent_steps_per_bench_step": n * T, "tuning": tuning},
        "final_invariants": {k: inv[k] for k in ("step", "n_s", "n_i", "n_r", "out_of_bounds",
                                                   "digest")},
        "runs_identical": h["same"],
        "kernels": kernels,
        "roofline": roof,
    }

    if not args.no_extra:
        out["extra"] = extras(torch, A)
        out["extra"]["paper_models"] = paper_models(torch, A)
        log(f"bench: extra {out['extra']}")
    if not args.no_big:
        h["bufs"] = None
        torch.cuda.empty_cache()
        out["roofline_big"] = roofline_big(torch, A, args.big_log2)
        log(f"bench: roofline_big {out['roofline_big']}")
    if not args.no_sweep:
        out["sweep"] = sweep_block(torch, A)
        log(f"bench: sweep {out['sweep']}")
    if args.serve:
        out["serve"] = serve_block(torch, A, args.serve, args.serve_scale, args.serve_budget_gib,
                                   args.serve_chunk)
        log(f"bench: serve {out['serve']}")
    if not args.no_cpu:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, args.cpu_sweep_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
