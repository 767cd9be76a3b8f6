"""ctypes wrapper of the plain C oracle ``amber_oracle.c`` (TEST INFRASTRUCTURE).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this.  The
arithmetic lives in the C file and in ``thresholds.py``; this module only
marshals numpy arrays.  Descriptor defaults (grid side, initial infected count)
are derived here from their definitions, independently of the GPU library.

Model statement followed: synchronous columnar updates (Sec. 3.4) of the three
benchmark models of Sec. 5.1.2, reformulated on an L x L torus grid with
counter-based Philox randomness; invariants of Sec. 5.1.3.
"""
import ctypes
import math
import os

import numpy as np

from . import thresholds

HERE = os.path.dirname(os.path.abspath(__file__))
# AMBER_ORACLE_LIB: another build of the same source (the sanitizer test)
LIB_PATH = os.environ.get("AMBER_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

WEALTH, RANDOM_WALK, SIR = 0, 1, 2
P_INIT_POS, P_MOVE, P_EPI, P_RECIPIENT = 0, 1, 2, 3

_lib = None

_u32 = ctypes.c_uint32
_i32 = ctypes.c_int32
_p = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_p, _u32, _u32, _p]
        L.orc_word.argtypes = [_u32] * 7
        L.orc_word.restype = _u32
        L.orc_recipient.argtypes = [_u32] * 5
        L.orc_recipient.restype = _u32
        L.orc_wealth_apply.argtypes = [_u32, _p, _p, _p]
        L.orc_neighbour_infected.argtypes = [_u32, _p, _i32, _i32]
        L.orc_neighbour_infected.restype = ctypes.c_uint64
        L.orc_digest.argtypes = [_u32, _u32, _p, _p]
        L.orc_digest.restype = ctypes.c_uint64
        L.orc_fmix64.argtypes = [ctypes.c_uint64]
        L.orc_fmix64.restype = ctypes.c_uint64
        L.orc_invariants.argtypes = [_u32, _u32, _p, _p, _p, _p, _p]
        L.orc_run_wealth.argtypes = [_u32, _i32, _u32, _u32, _u32, _u32, _p, ctypes.c_int]
        L.orc_run_walk.argtypes = [_u32, _u32, _u32, _u32, _u32, _u32, _p, _p, ctypes.c_int]
        L.orc_walk_agents.argtypes = [_u32, _p, _u32, _u32, _u32, _u32, _p, _p]
        L.orc_run_sir.argtypes = [_u32, _u32, _u32, _u32, _u32, _p, _u32, _u32,
                                  _u32, _u32, _p, _p, _p, ctypes.c_int]
        for f in (L.orc_run_wealth, L.orc_run_walk, L.orc_walk_agents, L.orc_run_sir):
            f.restype = ctypes.c_int
        u64 = ctypes.c_uint64
        L.orc_view_update_i32.argtypes = [u64, _p, _i32, _i32, _p, _p, ctypes.c_int, _i32,
                                          ctypes.c_float]
        L.orc_view_update_f32.argtypes = [u64, _p, ctypes.c_float, ctypes.c_float, _p, _p,
                                          ctypes.c_int, _i32, ctypes.c_float]
        L.orc_view_scatter_add_i32.argtypes = [u64, _p, u64, _p, _p, _i32]
        L.orc_view_scatter_add_f32.argtypes = [u64, _p, u64, _p, _p, ctypes.c_float]
        L.orc_view_write_log.argtypes = [u64, _p, u64, _p, _p]
        L.orc_grid_count.argtypes = [_u32, _p, u64, _p, _p, _u32, _p]
        L.orc_grid_neighbour_sum.argtypes = [_u32, _p, ctypes.c_int, ctypes.c_int, _p, _p]
        L.orc_grid_gather.argtypes = [_u32, _p, u64, _p, _p, _p]
        L.orc_graph_count.argtypes = [u64, _p, _p, _p, _u32, _p]
        L.orc_sir_transition.argtypes = [u64, _p, _p, _u32, _u32, _u32, _p, _u32, _u32]
        f32 = ctypes.c_float
        L.orc_cont_init.argtypes = [_u32, f32, _u32, _u32, _p, _p]
        L.orc_cont_walk.argtypes = [_u32, f32, _u32, _u32, _u32, _u32, _p, _p]
        L.orc_cont_sir.argtypes = [_u32, f32, f32, _u32, _u32, _p, _u32, _u32, _u32, _u32, _p, _p,
                                   _p, _p]
        L.orc_cont_sir.restype = ctypes.c_int
        L.orc_async_order.argtypes = [_u32, _u32, _u32, _u32, _p]
        L.orc_async_order.restype = ctypes.c_int
        L.orc_run_wealth_async.argtypes = [_u32, _u32, _u32, _u32, _u32, _p]
        L.orc_run_wealth_async.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


# ------------------------------------------------------------------ defaults

def grid_side(n: int) -> int:
    """round(sqrt(n)) with halves rounded up, in integers: s = isqrt(n) and
    L = s + 1 iff n > s^2 + s (i.e. sqrt(n) > s + 1/2)."""
    s = math.isqrt(n)
    return s + 1 if n > s * s + s else s


def default_initial_infected(n: int) -> int:
    """0.1% of the population, halves rounded up, at least one agent."""
    return max(1, (n + 500) // 1000)


# ------------------------------------------------------------------ random

def philox(ctr, k0: int, k1: int):
    c = np.array(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), k0, k1, _ptr(out))
    return [int(v) for v in out]


def word(seed, stream, purpose, words_per_agent, t, a, j):
    return int(lib().orc_word(seed, stream, purpose, words_per_agent, t, a, j))


def recipient(n, seed, stream, t, a):
    return int(lib().orc_recipient(n, seed, stream, t, a))


# ------------------------------------------------------------------ pieces

def wealth_apply(w, recip):
    """One synchronous transfer round with given recipients (donors: w > 0)."""
    w = np.array(w, dtype=np.int32)
    r = np.ascontiguousarray(recip, dtype=np.uint32)
    scratch = np.zeros_like(w)
    lib().orc_wealth_apply(len(w), _ptr(w), _ptr(r), _ptr(scratch))
    return w


def neighbour_infected(L, C, cx, cy):
    C = np.ascontiguousarray(C, dtype=np.uint32).reshape(-1)
    assert C.size == L * L
    return int(lib().orc_neighbour_infected(L, _ptr(C), cx, cy))


def digest(cols):
    """Order-free 64-bit digest of a population given its columns in order."""
    cols = [np.ascontiguousarray(c) for c in cols]
    n = len(cols[0])
    ptrs = (ctypes.c_void_p * len(cols))(*[c.ctypes.data for c in cols])
    widths = np.array([c.dtype.itemsize for c in cols], dtype=np.uint32)
    return int(lib().orc_digest(n, len(cols), ptrs, _ptr(widths)))


def fmix64(z):
    """SplitMix64's finaliser, as the digest uses it."""
    return int(lib().orc_fmix64(z & 0xFFFFFFFFFFFFFFFF))


class _Inv(ctypes.Structure):
    _fields_ = [("wealth_sum", ctypes.c_int64), ("wealth_min", ctypes.c_int32),
                ("n_s", ctypes.c_uint64), ("n_i", ctypes.c_uint64),
                ("n_r", ctypes.c_uint64), ("out_of_bounds", ctypes.c_uint64)]


def invariants(n, L=0, w=None, x=None, y=None, s=None):
    out = _Inv()
    lib().orc_invariants(n, L, _ptr(w), _ptr(x), _ptr(y), _ptr(s), ctypes.byref(out))
    return {f: getattr(out, f) for f, _ in _Inv._fields_}


# ------------------------------------------------------------------ view primitives

CMP = {"<": 0, "<=": 1, "==": 2, "!=": 3, ">=": 4, ">": 5}


def view_update(col, a, b, pred=None, cmp="<", thr=0):
    """Full view (pred None) or filtered view (rows where pred CMP thr, read
    before the update): v <- a*v + b, in place on a copy; returns the copy.
    int32 wraps modulo 2^32, float32 is one fused multiply-add."""
    col = np.array(col)
    assert col.dtype in (np.int32, np.float32)
    pi = pf = None
    if pred is not None:
        pred = np.ascontiguousarray(pred)
        if pred.dtype == np.int32:
            pi = pred
        elif pred.dtype == np.float32:
            pf = pred
        else:
            raise TypeError("predicate column must be int32 or float32")
        assert len(pred) == len(col)
    if col.dtype == np.int32:
        lib().orc_view_update_i32(len(col), _ptr(col), int(a), int(b), _ptr(pi), _ptr(pf),
                                  CMP[cmp], int(thr) if pi is not None else 0,
                                  float(thr) if pf is not None else 0.0)
    else:
        lib().orc_view_update_f32(len(col), _ptr(col), float(a), float(b), _ptr(pi), _ptr(pf),
                                  CMP[cmp], int(thr) if pi is not None else 0,
                                  float(thr) if pf is not None else 0.0)
    return col


def scatter_add(col, ids, vals=None, scalar=0):
    """Scatter view: for j in list order col[ids[j]] += vals[j] (or scalar);
    ids outside [0, len(col)) are skipped.  Returns the updated copy."""
    col = np.array(col)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=col.dtype)
        assert len(vals) == len(ids)
    if col.dtype == np.int32:
        lib().orc_view_scatter_add_i32(len(col), _ptr(col), len(ids), _ptr(ids), _ptr(vals),
                                       int(scalar))
    elif col.dtype == np.float32:
        lib().orc_view_scatter_add_f32(len(col), _ptr(col), len(ids), _ptr(ids), _ptr(vals),
                                       float(scalar))
    else:
        raise TypeError("column must be int32 or float32")
    return col


def write_log(col, ids, vals):
    """Buffered writes flushed once: in log order col[ids[j]] = vals[j] (the
    last write to an id stays); ids outside the column skipped.  int32 or
    float32 columns, values copied bit for bit.  Returns the updated copy."""
    col = np.array(col)
    assert col.dtype in (np.int32, np.float32)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=col.dtype)
    assert len(vals) == len(ids)
    lib().orc_view_write_log(len(col), _ptr(col), len(ids), _ptr(ids), _ptr(vals))
    return col


def _pos_array(pos):
    pos = [np.ascontiguousarray(p, dtype=np.int32) for p in pos]
    arr = (ctypes.c_void_p * len(pos))(*[p.ctypes.data for p in pos])
    return pos, arr


def grid_count(dims, pos, state=None, match=1):
    """Agents per cell of an n-D lattice (cell index with the first axis
    fastest), counting agents with state == match (all if state is None)."""
    dims = np.ascontiguousarray(dims, dtype=np.uint32)
    keep, arr = _pos_array(pos)
    out = np.zeros(int(np.prod(dims.astype(np.uint64))), dtype=np.uint32)
    st = None if state is None else np.ascontiguousarray(state, dtype=np.uint8)
    lib().orc_grid_count(len(dims), _ptr(dims), len(keep[0]), arr, _ptr(st), match, _ptr(out))
    return out


def grid_neighbour_sum(dims, counts, von_neumann=False, torus=True):
    dims = np.ascontiguousarray(dims, dtype=np.uint32)
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    out = np.zeros_like(counts)
    lib().orc_grid_neighbour_sum(len(dims), _ptr(dims), int(von_neumann), int(torus),
                                 _ptr(counts), _ptr(out))
    return out


def grid_gather(dims, pos, table):
    dims = np.ascontiguousarray(dims, dtype=np.uint32)
    keep, arr = _pos_array(pos)
    table = np.ascontiguousarray(table, dtype=np.uint32)
    out = np.zeros(len(keep[0]), dtype=np.uint32)
    lib().orc_grid_gather(len(dims), _ptr(dims), len(keep[0]), arr, _ptr(table), _ptr(out))
    return out


def graph_count(row, col, state, match=1):
    row = np.ascontiguousarray(row, dtype=np.uint32)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    state = np.ascontiguousarray(state, dtype=np.uint8)
    out = np.zeros(len(row) - 1, dtype=np.uint32)
    lib().orc_graph_count(len(row) - 1, _ptr(row), _ptr(col), _ptr(state), match, _ptr(out))
    return out


def sir_transition(state, k, seed, stream, t, beta=(1, 20), gamma=(1, 100)):
    s = np.array(state, dtype=np.uint8)
    k = np.ascontiguousarray(k, dtype=np.uint32)
    t_inf, k_sat = thresholds.infection_table(*beta)
    t_inf = np.array(t_inf, dtype=np.uint32)
    lib().orc_sir_transition(len(s), _ptr(s), _ptr(k), seed, stream, t, _ptr(t_inf), k_sat,
                             thresholds.recovery_threshold(*gamma))
    return s


class ContRun:
    """The paper's continuous-space models (Sec. 5.1.2) held on the host:
    model RANDOM_WALK (clamped walk) or SIR (contacts within radius r,
    probability p per contact, recovery after `recover` days), in a W x W
    world; float32 coordinates; ``step(k)`` advances steps t..t+k-1."""

    def __init__(self, model, n, W=100.0, r=5.0, seed=0, stream=0, p=(1, 10), recover=14,
                 initial_infected=5):
        self.model, self.n, self.W, self.r = model, n, float(W), float(r)
        self.seed, self.stream, self.recover, self.t = seed, stream, recover, 0
        self.x = np.zeros(n, dtype=np.float32)
        self.y = np.zeros(n, dtype=np.float32)
        lib().orc_cont_init(n, self.W, seed, stream, _ptr(self.x), _ptr(self.y))
        if model == SIR:
            self.s = np.zeros(n, dtype=np.uint8)
            self.s[:initial_infected] = 1
            self.days = np.zeros(n, dtype=np.uint8)
            t_inf, self.k_sat = thresholds.infection_table(*p)
            self.t_inf = np.array(t_inf, dtype=np.uint32)

    def step(self, k=1):
        if self.model == RANDOM_WALK:
            lib().orc_cont_walk(self.n, self.W, self.seed, self.stream, self.t, k, _ptr(self.x),
                                _ptr(self.y))
        else:
            rc = lib().orc_cont_sir(self.n, self.W, self.r, self.seed, self.stream,
                                    _ptr(self.t_inf), self.k_sat, self.recover, self.t, k,
                                    _ptr(self.x), _ptr(self.y), _ptr(self.s), _ptr(self.days))
            if rc != 0:
                raise RuntimeError("oracle cont_sir failed")
        self.t += k
        return self

    def columns(self):
        if self.model == RANDOM_WALK:
            return [self.x, self.y]
        return [self.x, self.y, self.s, self.days]


def async_order(n, seed, stream, t):
    """The acting order of step t under asynchronous semantics."""
    out = np.zeros(n, dtype=np.uint32)
    if lib().orc_async_order(n, seed, stream, t, _ptr(out)) != 0:
        raise RuntimeError("oracle async_order failed")
    return out


def run_wealth_async(w, seed, stream, t0, n_steps):
    """Wealth transfer with asynchronous (sequential) updates, steps
    t0..t0+n_steps-1 from the column w (copied)."""
    w = np.array(w, dtype=np.int32)
    if lib().orc_run_wealth_async(len(w), seed, stream, t0, n_steps, _ptr(w)) != 0:
        raise RuntimeError("oracle run_wealth_async failed")
    return w


# ------------------------------------------------------------------ runs

class OracleRun:
    """One simulation held on the host; ``step(k)`` advances steps t..t+k-1.

    Parameters mirror the GPU descriptor: model, n, grid side L (0 = round
    sqrt n), seed, stream, wealth_init, beta/gamma as num/den, initial
    infected (0 = default)."""

    def __init__(self, model, n, L=0, seed=0, stream=0, wealth_init=1,
                 beta=(1, 20), gamma=(1, 100), initial_infected=0):
        if n < 1:
            raise ValueError("n must be >= 1")
        self.model, self.n, self.seed, self.stream = model, n, seed, stream
        self.t = 0
        if model == WEALTH:
            self.L = 0
            self.w = np.zeros(n, dtype=np.int32)
            rc = lib().orc_run_wealth(n, wealth_init, seed, stream, 0, 0, _ptr(self.w), 1)
        elif model in (RANDOM_WALK, SIR):
            self.L = L if L else grid_side(n)
            self.x = np.zeros(n, dtype=np.int32)
            self.y = np.zeros(n, dtype=np.int32)
            if model == RANDOM_WALK:
                rc = lib().orc_run_walk(n, self.L, seed, stream, 0, 0,
                                        _ptr(self.x), _ptr(self.y), 1)
            else:
                self.i0 = initial_infected if initial_infected else default_initial_infected(n)
                self.t_inf, self.k_sat = thresholds.infection_table(*beta)
                self.t_inf = np.array(self.t_inf, dtype=np.uint32)
                self.t_rec = thresholds.recovery_threshold(*gamma)
                self.s = np.zeros(n, dtype=np.uint8)
                rc = self._sir(0, 0, 1)
        else:
            raise ValueError("unknown model")
        if rc != 0:
            raise RuntimeError("oracle init failed")

    @classmethod
    def resume(cls, model, columns, t, L=0, seed=0, stream=0, beta=(1, 20), gamma=(1, 100)):
        """A run continued from host columns holding its state after t steps
        (the columns are copied)."""
        self = cls.__new__(cls)
        self.model, self.seed, self.stream, self.t = model, seed, stream, t
        cols = [np.array(c) for c in columns]
        self.n = len(cols[0])
        if model == WEALTH:
            self.L = 0
            (self.w,) = [c.astype(np.int32) for c in cols]
        else:
            self.L = L if L else grid_side(self.n)
            self.x, self.y = cols[0].astype(np.int32), cols[1].astype(np.int32)
            if model == SIR:
                self.s = cols[2].astype(np.uint8)
                self.i0 = 0
                self.t_inf, self.k_sat = thresholds.infection_table(*beta)
                self.t_inf = np.array(self.t_inf, dtype=np.uint32)
                self.t_rec = thresholds.recovery_threshold(*gamma)
        return self

    def _sir(self, t0, k, do_init):
        return lib().orc_run_sir(self.n, self.L, self.seed, self.stream, self.i0,
                                 _ptr(self.t_inf), self.k_sat, self.t_rec, t0, k,
                                 _ptr(self.x), _ptr(self.y), _ptr(self.s), do_init)

    def step(self, k=1):
        if self.model == WEALTH:
            rc = lib().orc_run_wealth(self.n, 0, self.seed, self.stream, self.t, k,
                                      _ptr(self.w), 0)
        elif self.model == RANDOM_WALK:
            rc = lib().orc_run_walk(self.n, self.L, self.seed, self.stream, self.t, k,
                                    _ptr(self.x), _ptr(self.y), 0)
        else:
            rc = self._sir(self.t, k, 0)
        if rc != 0:
            raise RuntimeError("oracle step failed")
        self.t += k
        return self

    def columns(self):
        if self.model == WEALTH:
            return [self.w]
        if self.model == RANDOM_WALK:
            return [self.x, self.y]
        return [self.x, self.y, self.s]

    def digest(self):
        return digest(self.columns())

    def invariants(self):
        if self.model == WEALTH:
            return invariants(self.n, 0, w=self.w)
        if self.model == RANDOM_WALK:
            return invariants(self.n, self.L, x=self.x, y=self.y)
        return invariants(self.n, self.L, x=self.x, y=self.y, s=self.s)


def walk_agents(ids, L, seed, stream, n_steps):
    """Positions after n_steps of the listed random-walk agents, each replayed
    alone from its initial position."""
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    x = np.zeros(len(ids), dtype=np.int32)
    y = np.zeros(len(ids), dtype=np.int32)
    rc = lib().orc_walk_agents(len(ids), _ptr(ids), L, seed, stream, n_steps, _ptr(x), _ptr(y))
    if rc != 0:
        raise RuntimeError("oracle walk_agents failed")
    return x, y
