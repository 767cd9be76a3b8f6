"""Pure-Python brute force for tiny populations (TEST INFRASTRUCTURE).

Written independently of ``amber_oracle.c`` to pin it: its own Philox4x32-10,
per-agent dictionaries instead of columns, and an O(N^2) neighbour search that
tests torus distance instead of enumerating cells.  Use only for N up to a few
hundred agents and a few tens of steps.

Models follow Sec. 5.1.2 of the paper as reformulated on a torus grid, with
synchronous (snapshot) semantics (Sec. 3.4).
"""
from . import thresholds

MASK = 0xFFFFFFFF


def philox_block(c, key):
    """Philox4x32-10 (Salmon et al., SC'11) on a 4-word counter, 2-word key."""
    c = [v & MASK for v in c]
    k0, k1 = key[0] & MASK, key[1] & MASK
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & MASK
            k1 = (k1 + 0xBB67AE85) & MASK
        prod0 = 0xD2511F53 * c[0]
        prod1 = 0xCD9E8D57 * c[2]
        c = [((prod1 >> 32) ^ c[1] ^ k0) & MASK, prod1 & MASK,
             ((prod0 >> 32) ^ c[3] ^ k1) & MASK, prod0 & MASK]
    return c


PURPOSE = {"init_pos": (0, 2), "move": (1, 1), "epi": (2, 1), "recipient": (3, 2),
           "order": (4, 1), "step": (5, 2)}


def draw(seed, stream, purpose, t, a, j):
    p, words = PURPOSE[purpose]
    g = a * words + j
    return philox_block([g // 4, t, p, 0], [seed, stream])[g % 4]


MOVES = [(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1) if (dx, dy) != (0, 0)]


def coord(u, L):
    return (u * L) >> 32


def walker_init(n, L, seed, stream):
    return [{"x": coord(draw(seed, stream, "init_pos", 0, a, 0), L),
             "y": coord(draw(seed, stream, "init_pos", 0, a, 1), L)} for a in range(n)]


def move(agent, a, L, seed, stream, t):
    dx, dy = MOVES[draw(seed, stream, "move", t, a, 0) >> 29]
    agent["x"] = (agent["x"] + dx) % L
    agent["y"] = (agent["y"] + dy) % L


def wealth_run(n, w_init, seed, stream, steps):
    w = [w_init] * n
    for t in range(steps):
        donors = [a for a in range(n) if w[a] > 0]
        nw = list(w)
        for a in donors:
            u = (draw(seed, stream, "recipient", t, a, 0) << 32) | draw(seed, stream, "recipient", t, a, 1)
            r = (u * n) >> 64
            nw[a] -= 1
            nw[r] += 1
        w = nw
    return w


def wealth_run_async(w, seed, stream, t0, steps):
    """Asynchronous (sequential) semantics, Sec. 3.4: each step the agents act
    one at a time in the order of their ORDER draws (ties by id), each seeing
    the wealth as the agents before it left it."""
    w = list(w)
    n = len(w)
    for t in range(t0, t0 + steps):
        order = sorted(range(n), key=lambda a: (draw(seed, stream, "order", t, a, 0), a))
        for a in order:
            if w[a] > 0:
                u = (draw(seed, stream, "recipient", t, a, 0) << 32) | \
                    draw(seed, stream, "recipient", t, a, 1)
                w[a] -= 1
                w[(u * n) >> 64] += 1
    return w


def walk_run(n, L, seed, stream, steps):
    agents = walker_init(n, L, seed, stream)
    for t in range(steps):
        for a, ag in enumerate(agents):
            move(ag, a, L, seed, stream, t)
    return [ag["x"] for ag in agents], [ag["y"] for ag in agents]


def torus_near(u, v, L):
    """True iff cells u and v are within one step on a ring of L cells."""
    d = (u - v) % L
    return d in (0, 1, L - 1)


def sir_infected_neighbours(agents, states, a, L):
    """k for agent a: infected agents whose cell lies in the 3x3 torus block
    around a's cell, found by testing every agent (O(N) per query)."""
    me = agents[a]
    return sum(1 for j, other in enumerate(agents)
               if states[j] == 1 and torus_near(other["x"], me["x"], L)
               and torus_near(other["y"], me["y"], L))


def sir_run(n, L, seed, stream, steps, beta=(1, 20), gamma=(1, 100), i0=None,
            record=None):
    t_inf, k_sat = thresholds.infection_table(*beta)
    t_rec = thresholds.recovery_threshold(*gamma)
    if i0 is None:
        i0 = max(1, (n + 500) // 1000)
    agents = walker_init(n, L, seed, stream)
    states = [1 if a < i0 else 0 for a in range(n)]
    for t in range(steps):
        for a, ag in enumerate(agents):
            move(ag, a, L, seed, stream, t)
        new = list(states)
        for a in range(n):
            if states[a] == 0:
                k = sir_infected_neighbours(agents, states, a, L)
                if k and draw(seed, stream, "epi", t, a, 0) < t_inf[min(k, k_sat)]:
                    new[a] = 1
            elif states[a] == 1:
                if draw(seed, stream, "epi", t, a, 0) < t_rec:
                    new[a] = 2
        if record is not None:
            record.append(list(states))
        states = new
    return [ag["x"] for ag in agents], [ag["y"] for ag in agents], states


def cont_run(model, n, W, r, seed, stream, steps, p=(1, 10), recover=14, i0=5):
    """The continuous-space walk ("walk") or SIR ("sir") of Sec. 5.1.2 with
    numpy float32 scalars (every operation rounds to float32) and an
    all-pairs contact test written as a distance check per pair."""
    import numpy as np
    f = np.float32
    W = f(W)

    def unit(u, scale):
        return f(u >> 8) * f(scale)

    xs = [unit(draw(seed, stream, "init_pos", 0, a, 0), 2.0 ** -24) * W for a in range(n)]
    ys = [unit(draw(seed, stream, "init_pos", 0, a, 1), 2.0 ** -24) * W for a in range(n)]
    state = [1 if a < i0 else 0 for a in range(n)]
    days = [0] * n
    table, k_sat = thresholds.infection_table(*p)
    r2 = f(r) * f(r)
    for t in range(steps):
        for a in range(n):
            dx = unit(draw(seed, stream, "step", t, a, 0), 2.0 ** -23) - f(1)
            dy = unit(draw(seed, stream, "step", t, a, 1), 2.0 ** -23) - f(1)
            xs[a] = min(max(xs[a] + dx, f(0)), W)
            ys[a] = min(max(ys[a] + dy, f(0)), W)
        if model == "walk":
            continue
        before = list(state)
        for a in range(n):
            if before[a] == 0:
                k = 0
                for b in range(n):
                    if before[b] == 1:
                        ddx, ddy = xs[a] - xs[b], ys[a] - ys[b]
                        if ddx * ddx + ddy * ddy <= r2:
                            k += 1
                if k and draw(seed, stream, "epi", t, a, 0) < table[min(k, k_sat)]:
                    state[a], days[a] = 1, 0
            elif before[a] == 1:
                days[a] += 1
                if days[a] >= recover:
                    state[a] = 2
    return xs, ys, state, days
