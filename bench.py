"""Benchmark of the columnar ABM hot path on one MI355X.

Workload (the metric's headline case): grid SIR with N = 1e6 agents on a
1000 x 1000 torus, beta = 1/20, gamma = 1/100, 0.1% initially infected,
key (0, 0); 500 steps in total = W untimed warm-up steps followed by K timed
steps (defaults W = 20, K = 480).  One bench step = one model step of the whole
population (move, cell binning, neighbour count, transitions), all on the GPU.

Prints ONE JSON line: agent-steps/s over the K timed steps, the roofline of the
dominant kernel (algorithmic bytes per launch / average launch time, HIP events
on the library's stream), the CPU oracle timed on a bounded sample, and extra
lines for the wealth and random-walk models.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
                  [--no-sweep] [--serve N [--serve-scale S] [--serve-plain]]
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
                  for f in ("amber_device.hip", "amber_device_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")


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
    1 .. len-1 of each call).  counts[k] = (S, I) at the start of timed step
    k.  Launch j is the first of its call with S = 0 three steps back; it
    runs every remaining step of the call in registers (one pass over the
    columns, 18 B/agent), and the later launches of the call move nothing."""
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
    """Bytes one step of the tiled SIR mode must move: each agent's 8-byte
    record read and written, and the L*L count grid written and read once."""
    return 16 * n + 8 * L * L


def wealth_step_bytes(n, donors):
    """Wealth read and written (8 B per agent) plus one 8-B RMW per donor."""
    return 8 * n + 8 * donors


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


def sir_bench(torch, A, W, K, chunk, form, count=0, tuning=None, block=256, tile=0):
    from paper_2601_16292_amd import workloads as WL
    c = WL.SIR_1M

    def mk():
        p = A.Population(A.SIR, c["n"], L=c["L"], seed=c["seed"], stream_id=c["stream"],
                         beta=c["beta"], gamma=c["gamma"])
        if tuning:
            p.tune(**tuning)
        else:
            p.tune(block=block, sir_form=form, sir_count=count, sir_tile=tile)
        return p

    pop = mk()
    pop.step(W)
    secs = timed_steps(torch, pop, K, chunk)
    inv = pop.invariants()
    pop.release()

    # instrumented replay of the same steps: per-kernel launch times
    pop = mk()
    pop.step(W)
    torch.cuda.synchronize()
    pop.profile(True)
    done = 0
    while done < K:
        cc = min(chunk or K, K - done)
        pop.step(cc)
        done += cc
    times = pop.kernel_times()
    pop.release()

    # susceptible and infected counts at the start of every timed step (for
    # the grid's and the atomics' bytes)
    pop = mk()
    pop.step(W)
    counts = []
    for _ in range(K):
        v = pop.invariants()
        counts.append((v["n_s"], v["n_i"]))
        pop.step(1)
    pop.release()
    return secs, inv, times, counts


def roofline_for(times, bytes_per_kernel_total, traffic):
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
           "avg_launch_us": round(avg_s * 1e6, 3),
           "algorithmic_bytes_per_launch": int(bytes_per_launch)}
    if traffic and traffic.get("kernel") == name:
        # the number of launches of a call can vary (the host stops enqueueing
        # once one launch has run the call's remaining steps): bytes of the
        # whole call over this run's launches
        if "bytes_per_call" in traffic:
            out["traffic"] = int(traffic["bytes_per_call"] / launches)
        else:
            out["traffic"] = traffic.get("bytes_per_launch")
    return out


def load_traffic():
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    valid only if the kernel source has not changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t


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


def cpu_baseline(budget_s):
    """The oracle (single-threaded C), timed on the host on a bounded prefix of
    the same SIR workload: steps 0, 1, 2, ... until the budget is spent."""
    from oracle import oracle as O
    from paper_2601_16292_amd import workloads as WL
    c = WL.SIR_1M
    r = O.OracleRun(O.SIR, c["n"], c["L"], seed=c["seed"], stream=c["stream"], beta=c["beta"],
                    gamma=c["gamma"])
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < budget_s and steps < c["steps"]:
        r.step(1)
        steps += 1
    secs = time.perf_counter() - t0
    return {"value": round(c["n"] * steps / secs, 1), "unit": "agent-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"grid SIR N=1e6 L=1000, steps 0..{steps - 1} of 500 from init "
                      f"({secs:.1f} s, single-threaded C oracle, -O2)",
            "host_cpus": os.cpu_count()}


def roofline_big(torch, A, log2n):
    """Per-step kernels at an out-of-cache size (columns far above the 256 MB
    last-level cache): average launch time from HIP events on the library's
    stream, algorithmic bytes per launch, achieved GB/s against HBM peak."""
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

    # wealth, partition exchange at 2^24 agents (its largest size): 8 B per
    # agent + 8 B per donor in one launch per step
    nx = 1 << 24
    pop = A.Population(A.WEALTH, nx, wealth_init=1)
    pop.tune(wealth_form=2)
    pop.step(2)
    (w,) = pop.read()
    donors = int((w > 0).sum())
    del w
    pop.profile(True)
    pop.step(3)
    res["wealth_exchange_2p24"] = priced("wealth_exchange", pop.kernel_times(), 8 * nx + 8 * donors)
    res["wealth_exchange_2p24"]["donors_first_step"] = donors
    pop.release()
    torch.cuda.empty_cache()

    # wealth at n: partition exchange (2^15-agent partitions) and the global
    # atomic scatter; 8 B per agent + 8 B per donor
    for form, name, label in ((2, "wealth_exchange", "wealth_exchange"),
                              (1, "wealth_step", "wealth_step")):
        pop = A.Population(A.WEALTH, n, wealth_init=1)
        pop.tune(wealth_form=form)
        pop.step(2)
        (w,) = pop.read()
        donors = int((w > 0).sum())
        del w
        pop.profile(True)
        pop.step(3)
        res[label] = priced(name, pop.kernel_times(), 8 * n + 8 * donors)
        res[label]["donors_after_step_2"] = donors
        pop.release()
        torch.cuda.empty_cache()

    # SIR pipelined body: 18 B per agent + 8 B per cell + 8 B per infected,
    # in both count modes (gather: the body reads the 3x3 block of the count
    # grid; box: a stencil kernel box-sums the grid, the body reads one cell)
    for mode, label in ((1, "gather"), (2, "box")):
        pop = A.Population(A.SIR, n, L=0, beta=(1, 20), gamma=(1, 100))
        L = pop.info().grid_side
        pop.tune(sir_form=1, sir_count=mode)
        pop.step(30)
        i_t = pop.invariants()["n_i"]
        pop.profile(True)
        pop.step(2)        # the body is step 31
        times = pop.kernel_times()
        step_bytes = 18 * n + 8 * L * L + 8 * i_t
        if mode == 1:
            entry = priced("sir_body", times, step_bytes)
        else:
            entry = priced("sir_body_box", times, step_bytes - 8 * L * L)
            entry["box_kernel"] = priced("sir_box", {"sir_box": (times["sir_box"][0],
                                                                 times["sir_box"][1])},
                                         8 * L * L)
            both = (times["sir_body_box"][1] / times["sir_body_box"][0] +
                    times["sir_box"][1] / times["sir_box"][0]) / 1e3
            entry["step_GBs"] = round(step_bytes / both / 1e9, 1)
            entry["step_frac_of_hbm_peak"] = round(step_bytes / both / 1e9 / PEAK_HBM_GBS, 4)
        entry.update({"grid_side": L, "infected": i_t})
        res[f"sir_body_{label}"] = entry
        pop.release()
        torch.cuda.empty_cache()

    # SIR tiled mode: records sorted by tile, counts in LDS.  Priced on the
    # bytes it must move (16 B per agent, 8 B per cell); step_GBs prices the
    # same launch with the method's algorithmic bytes, as for the other modes
    for tile in (32, 64):
        pop = A.Population(A.SIR, n, L=0, beta=(1, 20), gamma=(1, 100))
        L = pop.info().grid_side
        pop.tune(sir_form=1, sir_count=4, sir_tile=tile)
        pop.step(30)
        i_t = pop.invariants()["n_i"]
        pop.profile(True)
        pop.step(2)        # the body is step 31
        times = pop.kernel_times()
        entry = priced("sir_tile_body", times, tile_step_bytes(n, L))
        step_bytes = 18 * n + 8 * L * L + 8 * i_t
        avg = times["sir_tile_body"][1] / times["sir_tile_body"][0] / 1e3
        entry["step_GBs"] = round(step_bytes / avg / 1e9, 1)
        entry["step_frac_of_hbm_peak"] = round(step_bytes / avg / 1e9 / PEAK_HBM_GBS, 4)
        entry["call_kernels_us"] = {k: round(v[1] / max(1, v[0]) * 1e3, 1) for k, v in times.items()}
        entry.update({"grid_side": L, "infected": i_t, "tile": tile})
        res[f"sir_body_tiled{tile}"] = entry
        pop.release()
        torch.cuda.empty_cache()

    # a whole SIR run at this size: 499 steps in one call after one step, in
    # the automatic mode (tiled, then gather once few susceptible agents are
    # left), all in the gather mode, and all in the tiled mode
    runs = {}
    for label, tu in (("auto", {}), ("gather", dict(sir_form=1, sir_count=1)),
                      ("tiled32", dict(sir_form=1, sir_count=4, sir_tile=32))):
        pop = A.Population(A.SIR, n, L=0, beta=(1, 20), gamma=(1, 100))
        if tu:
            pop.tune(**tu)
        pop.step(1)
        secs = timed_steps(torch, pop, 499, 0)
        inv = pop.invariants()
        runs[label] = {"seconds": round(secs, 4), "agent_steps_per_s": round(n * 499 / secs, 1),
                       "digest": inv["digest"]}
        pop.release()
        torch.cuda.empty_cache()
    runs["identical_outputs"] = (runs["auto"]["digest"] == runs["gather"]["digest"]
                                 == runs["tiled32"]["digest"])
    res["sir_whole_run_499_steps"] = runs
    return res


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
    ap.add_argument("--steps", type=int, default=480)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--chunk", type=int, default=0, help="steps per amber_step call (0 = all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--sir-form", choices=["auto", "pipelined", "persistent"], default="auto")
    ap.add_argument("--sir-count", choices=["auto", "gather", "box", "exchange", "tiled"],
                    default="auto")
    ap.add_argument("--sir-tile", type=int, default=0, choices=[0, 32, 64],
                    help="tile side of the tiled count mode (0 = automatic)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="use --sir-form/--sir-count instead of the autotuner's choice")
    ap.add_argument("--block", type=int, default=256,
                    help="threads per workgroup when --no-autotune is given")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 256-replicate sweep")
    ap.add_argument("--roofline-big", action="store_true",
                    help="also time the per-step kernels at an out-of-cache size")
    ap.add_argument("--big-log2", type=int, default=27)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve", type=int, default=0,
                    help="serve the first N requests of the 10,000-request stream (0 = skip)")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="arrival clock speed-up (1 = Poisson 50/s in real time)")
    ap.add_argument("--serve-budget-gib", type=float, default=200.0)
    ap.add_argument("--serve-chunk", type=int, default=50)
    ap.add_argument("--serve-plain", action="store_true",
                    help="also serve the stream FIFO one request at a time")
    args = ap.parse_args()

    if args.copy_probe:
        copy_probe()
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(runs and replicates are independent; see the sharding design notes). "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.warmup + args.steps > 0xFFFFFFFF or args.steps < 1:
        sys.exit("bad --steps/--warmup")

    import torch
    from paper_2601_16292_amd import amber as A
    A.lib()
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    torch.cuda.set_device(0)

    n, L = 1_000_000, 1000
    form = {"auto": 0, "pipelined": 1, "persistent": 2}[args.sir_form]
    count = {"auto": 0, "gather": 1, "box": 2, "exchange": 3, "tiled": 4}[args.sir_count]
    log(f"bench: SIR N={n} L={L} warmup={args.warmup} steps={args.steps} form={args.sir_form} "
        f"count={args.sir_count}")
    tuning = None
    if args.autotune:
        from paper_2601_16292_amd import autotune as AT
        tuning = AT.tune(A.SIR, n, L=L, steps=args.steps, warmup=args.warmup, torch=torch,
                         force=True, log=log)
        log(f"bench: autotuned {tuning}")
    secs, inv, times, counts = sir_bench(torch, A, args.warmup, args.steps, args.chunk, form,
                                         count, tuning, args.block, args.sir_tile)
    value = n * args.steps / secs
    log(f"bench: {value:.4g} agent-steps/s, {secs * 1e3 / args.steps:.4f} ms/step, kernels {times}")

    # algorithmic bytes per launch of each SIR kernel over the timed steps
    calls = [min(args.chunk or args.steps, args.steps - a)
             for a in range(0, args.steps, args.chunk or args.steps)]
    step_bytes = [sir_step_bytes(n, L, i_t, s_t) for s_t, i_t in counts]
    region_bytes = sum(step_bytes)
    priced = {}
    if "sir_persistent" in times:
        priced["sir_persistent"] = sum(step_bytes)          # every step in each launch
    if "sir_body" in times:                                 # gather mode, one step per launch
        priced["sir_body"] = sir_gather_body_bytes(n, L, counts, calls)
        heads = [sum(calls[:c]) for c in range(len(calls))]
        region_bytes = priced["sir_body"] + sum(step_bytes[a] for a in heads)
    live = [s_t > 0 for s_t, _ in counts]                  # steps that read counts
    cols = [18 * n + (8 * i_t if s_t else 0) for s_t, i_t in counts]
    if "sir_xbody" in times:                                # exchange mode: grid bytes go to sir_xcount
        priced["sir_xbody"] = sum(cols)
        priced["sir_xcount"] = 8 * L * L * sum(live)
    if "sir_tile_body" in times:
        # tiled mode keeps 8-byte records instead of the columns: priced on the
        # bytes it must move (records read and written, count grid written and read)
        priced["sir_tile_body"] = sum(16 * n + (8 * L * L if v else 0) for v in live[1:])
    if "sir_body_box" in times:                             # box mode: grid bytes go to sir_box
        priced["sir_body_box"] = sum(cols[1:])
        priced["sir_box"] = 8 * L * L * sum(live)
    roof = roofline_for(times, priced, load_traffic())
    if roof is not None:
        roof["timed_region_GBs"] = round(region_bytes / secs / 1e9, 1)
        if roof["kernel"] == "sir_body":
            roof["limits"] = ("by phase: global atomics while every infected agent is binned; "
                              "dependent byte loads with demand-driven binning; Philox VALU "
                              "work in the launch that finishes the call "
                              "(profiles/sir_1m_phase_counters.md)")
    kernels = {k: {"launches": v[0], "avg_us": round(v[1] / max(1, v[0]) * 1e3, 3)}
               for k, v in times.items()}

    out = {
        "metric": "agent-steps/sec (1e6-agent SIR, wealth); sweep p50/p99 latency, batched vs plain",
        "value": round(value, 1),
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded Philox initial state; no dataset)",
        "config": {"workload": "grid SIR, N=1e6 on a 1000x1000 torus, beta=1/20, gamma=1/100, "
                               "0.1% initially infected, key (0,0), 500 steps",
                   "n_agents": n, "grid_side": L, "timed_steps": f"{args.warmup}..{args.warmup + args.steps - 1}",
                   "chunk": args.chunk or args.steps,
                   "tuning": tuning if tuning else {"sir_form": args.sir_form,
                                                     "sir_count": args.sir_count,
                                                     "sir_tile": args.sir_tile,
                                                     "block": args.block}},
        "final_invariants": {k: inv[k] for k in ("step", "n_s", "n_i", "n_r", "digest")},
        "kernels": kernels,
        "roofline": roof,
    }

    if not args.no_extra:
        extra = {}
        s, winv = wealth_bench(torch, A, 1000, 0, 100)
        extra["wealth_1k"] = {"value": round(1000 * 100 / s, 1), "unit": "agent-steps/s",
                              "steps": 100, "ms_total": round(s * 1e3, 4),
                              "wealth_sum": winv["wealth_sum"]}
        for form, label in ((0, "wealth_1m"), (1, "wealth_1m_atomic")):
            s, winv = wealth_bench(torch, A, 1_000_000, 10, 200, form=form)
            extra[label] = {"value": round(1e6 * 200 / s, 1), "unit": "agent-steps/s",
                            "steps": 200, "ms_per_step": round(s * 1e3 / 200, 5),
                            "wealth_sum": winv["wealth_sum"]}
        if args.sir_form == "auto":
            s2, _, t2, _ = sir_bench(torch, A, args.warmup, args.steps, args.chunk, 1, 1)
            extra["sir_1m_pipelined_gather"] = {"value": round(n * args.steps / s2, 1),
                                         "unit": "agent-steps/s",
                                         "ms_per_step": round(s2 * 1e3 / args.steps, 5),
                                         "kernels": {k: {"launches": v[0],
                                                         "avg_us": round(v[1] / max(1, v[0]) * 1e3, 3)}
                                                     for k, v in t2.items()}}
        s, rinv = walk_bench(torch, A, 1_000_000, 1000, 1000)
        extra["walk_1m"] = {"value": round(1e6 * 1000 / s, 1), "unit": "agent-steps/s",
                            "steps": 1000, "ms_total": round(s * 1e3, 4),
                            "out_of_bounds": rinv["out_of_bounds"]}
        out["extra"] = extra
        log(f"bench: extra {extra}")

    if args.roofline_big:
        out["roofline_big"] = roofline_big(torch, A, args.big_log2)
        log(f"bench: roofline_big {out['roofline_big']}")

    if not args.no_sweep:
        from paper_2601_16292_amd import sweep as SW, workloads as WL
        runs = WL.sir_sweep()
        log(f"bench: sweep of {len(runs)} SIR replicates, sum N = {sum(r['n'] for r in runs)}")
        forms = {"plain": SW.run_plain(runs, torch), "batched": SW.run_batched(runs, torch),
                 "batched_graph": SW.run_batched(runs, torch, graph=True)}
        same = forms["plain"]["digests"] == forms["batched"]["digests"] == forms["batched_graph"]["digests"]
        out["sweep"] = {k: {"value": round(v["value"], 1), "unit": "agent-steps/s",
                            "seconds": round(v["seconds"], 4), "p50_s": round(v["p50_s"], 4),
                            "p99_s": round(v["p99_s"], 4)} for k, v in forms.items()}
        out["sweep"]["identical_outputs"] = bool(same)
        out["sweep"]["workload"] = ("256 SIR replicates, N log-uniform in [1e3, 1e6], grid side "
                                    "round(sqrt N), beta 16 values 0.01..0.2, gamma 1/100, 300 steps, "
                                    "key (0, r); latency from sweep submission")
        log(f"bench: sweep {out['sweep']}")

    if args.serve:
        from paper_2601_16292_amd import serve as SV, workloads as WL
        reqs = WL.served_stream()[:args.serve]
        log(f"bench: served stream of {len(reqs)} requests, time scale {args.serve_scale}")
        served = SV.serve([dict(r) for r in reqs], budget_bytes=int(args.serve_budget_gib * 2**30),
                          chunk=args.serve_chunk, time_scale=args.serve_scale, log=log)
        entry = {"served": {k: served[k] for k in ("requests", "agent_steps", "seconds", "p50_s",
                                                   "p99_s", "ticks")},
                 "time_scale": args.serve_scale, "budget_gib": args.serve_budget_gib,
                 "chunk": args.serve_chunk}
        entry["served"]["value"] = round(served["value"], 1)
        if args.serve_plain:
            plain = SV.serve_plain([dict(r) for r in reqs], time_scale=args.serve_scale, log=log)
            entry["plain"] = {k: plain[k] for k in ("requests", "agent_steps", "seconds", "p50_s",
                                                    "p99_s")}
            entry["plain"]["value"] = round(plain["value"], 1)
            da = {r["id"]: r["digest"] for r in served["records"]}
            db = {r["id"]: r["digest"] for r in plain["records"]}
            entry["identical_outputs"] = da == db
        out["serve"] = entry
        log(f"bench: serve {entry}")

    if not args.no_cpu:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
