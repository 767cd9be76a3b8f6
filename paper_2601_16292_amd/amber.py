"""ctypes binding of libamber (include/amber.h): argument marshalling only.

Every function mirrors the C entry point of the same name and returns its
status code; ``check`` turns a non-zero status into ``AmberError`` with the
library's message.  ``Population`` is a convenience owner of the device
buffers one run needs (PyTorch tensors on the current device) and of the
handle; every step of the path runs in the library's HIP kernels.

There is no CPU fallback: loading fails loudly when ``libamber.so`` is
missing.
"""
import atexit
import ctypes
import os
import weakref

PKG = os.path.dirname(os.path.abspath(__file__))
# AMBER_LIB_PATH: another build of the same sources (the host-sanitizer test)
LIB_PATH = os.environ.get("AMBER_LIB_PATH") or os.path.join(PKG, "libamber.so")

ABI_VERSION = 1
MAX_TABLE = 8192

WEALTH, RANDOM_WALK, SIR = 0, 1, 2
COL_WEALTH, COL_X, COL_Y, COL_STATE = 0, 1, 2, 3
NUM_COLS = 4

OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "AMBER_OK", -1: "AMBER_E_INVALID", -2: "AMBER_E_NOMEM",
                -3: "AMBER_E_DEVICE", -4: "AMBER_E_STATE", -5: "AMBER_E_UNSUPPORTED"}

MODEL_COLUMNS = {WEALTH: [COL_WEALTH], RANDOM_WALK: [COL_X, COL_Y],
                 SIR: [COL_X, COL_Y, COL_STATE]}

EXPORTED = ["amber_abi_version", "amber_column_bytes", "amber_workspace_bytes",
            "amber_infection_table", "amber_init_population",
            "amber_init_population_noalloc", "amber_resume_population",
            "amber_view_update", "amber_view_scatter_workspace_bytes",
            "amber_view_scatter_add", "amber_view_write_log_workspace_bytes",
            "amber_view_write_log", "amber_async_workspace_bytes", "amber_step_async",
            "amber_grid_count", "amber_grid_neighbour_sum", "amber_grid_gather",
            "amber_graph_neighbour_count", "amber_sir_transition", "amber_recovery_threshold",
            "amber_cont_init", "amber_cont_walk", "amber_cont_sir_workspace_bytes",
            "amber_cont_sir", "amber_step",
            "amber_step_batch", "amber_read_columns", "amber_invariants",
            "amber_pop_info", "amber_set_tuning", "amber_get_tuning",
            "amber_profile_enable", "amber_profile_read",
            "amber_release", "amber_last_error"]


class RunDesc(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("model", ctypes.c_uint32),
                ("n_agents", ctypes.c_uint32), ("grid_side", ctypes.c_uint32),
                ("seed", ctypes.c_uint32), ("stream", ctypes.c_uint32),
                ("wealth_init", ctypes.c_int32),
                ("beta_num", ctypes.c_uint32), ("beta_den", ctypes.c_uint32),
                ("gamma_num", ctypes.c_uint32), ("gamma_den", ctypes.c_uint32),
                ("initial_infected", ctypes.c_uint32)]


class Buffers(ctypes.Structure):
    _fields_ = [("col", ctypes.c_void_p * NUM_COLS), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class Invariants(ctypes.Structure):
    _fields_ = [("step", ctypes.c_uint64), ("wealth_sum", ctypes.c_int64),
                ("wealth_min", ctypes.c_int32), ("reserved0", ctypes.c_uint32),
                ("n_s", ctypes.c_uint64), ("n_i", ctypes.c_uint64), ("n_r", ctypes.c_uint64),
                ("out_of_bounds", ctypes.c_uint64), ("digest", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved0"}


class PopInfo(ctypes.Structure):
    _fields_ = [("model", ctypes.c_uint32), ("n_agents", ctypes.c_uint32),
                ("grid_side", ctypes.c_uint32), ("initial_infected", ctypes.c_uint32),
                ("seed", ctypes.c_uint32), ("stream", ctypes.c_uint32),
                ("table_len", ctypes.c_uint32), ("t_rec", ctypes.c_uint32),
                ("step", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("sir_form", ctypes.c_uint32),
                ("max_groups_per_thread", ctypes.c_uint32), ("sir_count", ctypes.c_uint32),
                ("wealth_form", ctypes.c_uint32), ("sir_tile", ctypes.c_uint32),
                ("sir_poll", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


SIR_AUTO, SIR_PIPELINED, SIR_PERSISTENT = 0, 1, 2
COUNT_AUTO, COUNT_GATHER, COUNT_BOX, COUNT_EXCHANGE, COUNT_TILED, COUNT_TILED_GATHER = 0, 1, 2, 3, 4, 5
WEALTH_AUTO, WEALTH_ATOMIC, WEALTH_EXCHANGE, WEALTH_EXCHANGE_WIDE = 0, 1, 2, 3
POLL_NOWAIT, POLL_OFF, POLL_PACED = 0, 1, 2


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double)]


DT_I32, DT_F32 = 0, 1
CMP = {"<": 0, "<=": 1, "==": 2, "!=": 3, ">=": 4, ">": 5}


class Value(ctypes.Union):
    _fields_ = [("i", ctypes.c_int32), ("f", ctypes.c_float)]


def value(dtype, v):
    out = Value()
    if dtype == DT_I32:
        out.i = int(v)
    else:
        out.f = float(v)
    return out


class AmberError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libamber.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # Load PyTorch's HIP runtime first when it is installed, so that the
        # library and torch share one runtime (and one notion of streams).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.amber_abi_version.restype = ctypes.c_uint32
        L.amber_abi_version.argtypes = []
        L.amber_column_bytes.restype = ctypes.c_size_t
        L.amber_column_bytes.argtypes = [ctypes.POINTER(RunDesc), ctypes.c_int]
        L.amber_workspace_bytes.restype = ctypes.c_size_t
        L.amber_workspace_bytes.argtypes = [ctypes.POINTER(RunDesc)]
        L.amber_infection_table.restype = ctypes.c_int
        L.amber_infection_table.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P,
                                            ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        L.amber_init_population.restype = ctypes.c_int
        L.amber_init_population.argtypes = [ctypes.POINTER(RunDesc), ctypes.POINTER(Buffers),
                                            P, ctypes.POINTER(P)]
        L.amber_init_population_noalloc.restype = ctypes.c_int
        L.amber_init_population_noalloc.argtypes = [ctypes.POINTER(RunDesc),
                                                    ctypes.POINTER(Buffers), P,
                                                    ctypes.POINTER(P)]
        L.amber_resume_population.restype = ctypes.c_int
        L.amber_resume_population.argtypes = [ctypes.POINTER(RunDesc), ctypes.POINTER(Buffers),
                                              ctypes.POINTER(P), ctypes.c_uint64, P,
                                              ctypes.POINTER(P)]
        L.amber_view_update.restype = ctypes.c_int
        L.amber_view_update.argtypes = [P, ctypes.c_uint32, ctypes.c_uint64, Value, Value, P,
                                        ctypes.c_uint32, ctypes.c_uint32, Value, P]
        L.amber_view_scatter_workspace_bytes.restype = ctypes.c_size_t
        L.amber_view_scatter_workspace_bytes.argtypes = [ctypes.c_uint32, ctypes.c_uint64,
                                                         ctypes.c_uint64]
        L.amber_view_scatter_add.restype = ctypes.c_int
        L.amber_view_scatter_add.argtypes = [P, ctypes.c_uint32, ctypes.c_uint64, P,
                                             ctypes.c_uint64, P, Value, P, ctypes.c_size_t, P]
        L.amber_view_write_log_workspace_bytes.restype = ctypes.c_size_t
        L.amber_view_write_log_workspace_bytes.argtypes = [ctypes.c_uint64]
        L.amber_view_write_log.restype = ctypes.c_int
        L.amber_view_write_log.argtypes = [P, ctypes.c_uint32, ctypes.c_uint64, P,
                                           ctypes.c_uint64, P, P, ctypes.c_size_t, P]
        L.amber_async_workspace_bytes.restype = ctypes.c_size_t
        L.amber_async_workspace_bytes.argtypes = [ctypes.POINTER(RunDesc)]
        L.amber_step_async.restype = ctypes.c_int
        L.amber_step_async.argtypes = [P, ctypes.c_uint32, P, ctypes.c_size_t]
        PP = ctypes.POINTER(P)
        U32P = ctypes.POINTER(ctypes.c_uint32)
        u32, u64 = ctypes.c_uint32, ctypes.c_uint64
        L.amber_grid_count.restype = ctypes.c_int
        L.amber_grid_count.argtypes = [PP, u32, U32P, u64, P, u32, P, P]
        L.amber_grid_neighbour_sum.restype = ctypes.c_int
        L.amber_grid_neighbour_sum.argtypes = [P, u32, U32P, u32, u32, P, P]
        L.amber_grid_gather.restype = ctypes.c_int
        L.amber_grid_gather.argtypes = [P, PP, u32, U32P, u64, P, P]
        L.amber_graph_neighbour_count.restype = ctypes.c_int
        L.amber_graph_neighbour_count.argtypes = [P, P, u64, u64, P, u32, P, P]
        L.amber_sir_transition.restype = ctypes.c_int
        L.amber_sir_transition.argtypes = [P, P, u64, u32, u32, u32, P, u32, u32, P]
        L.amber_recovery_threshold.restype = ctypes.c_int
        L.amber_recovery_threshold.argtypes = [u32, u32, ctypes.POINTER(ctypes.c_uint32)]
        f32 = ctypes.c_float
        L.amber_cont_init.restype = ctypes.c_int
        L.amber_cont_init.argtypes = [P, P, P, P, u64, f32, u32, u32, u32, P]
        L.amber_cont_walk.restype = ctypes.c_int
        L.amber_cont_walk.argtypes = [P, P, u64, f32, u32, u32, u32, u32, P]
        L.amber_cont_sir_workspace_bytes.restype = ctypes.c_size_t
        L.amber_cont_sir_workspace_bytes.argtypes = [u64, f32, f32, u32, u32]
        L.amber_cont_sir.restype = ctypes.c_int
        L.amber_cont_sir.argtypes = [P, P, P, P, u64, f32, f32, u32, u32, u32, u32, u32, u32, u32,
                                     P, ctypes.c_size_t, P]
        L.amber_step.restype = ctypes.c_int
        L.amber_step.argtypes = [P, ctypes.c_uint32]
        L.amber_step_batch.restype = ctypes.c_int
        L.amber_step_batch.argtypes = [ctypes.POINTER(P), ctypes.c_uint32, ctypes.c_uint32]
        L.amber_read_columns.restype = ctypes.c_int
        L.amber_read_columns.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(P)]
        L.amber_invariants.restype = ctypes.c_int
        L.amber_invariants.argtypes = [P, ctypes.POINTER(Invariants)]
        L.amber_pop_info.restype = ctypes.c_int
        L.amber_pop_info.argtypes = [P, ctypes.POINTER(PopInfo)]
        L.amber_set_tuning.restype = ctypes.c_int
        L.amber_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.amber_get_tuning.restype = ctypes.c_int
        L.amber_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.amber_profile_enable.restype = ctypes.c_int
        L.amber_profile_enable.argtypes = [P, ctypes.c_int]
        L.amber_profile_read.restype = ctypes.c_int
        L.amber_profile_read.argtypes = [P, ctypes.POINTER(KernelTime), ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_uint32)]
        L.amber_release.restype = ctypes.c_int
        L.amber_release.argtypes = [P]
        L.amber_last_error.restype = ctypes.c_char_p
        L.amber_last_error.argtypes = []
        _lib = L
    return _lib


def amber_last_error():
    return lib().amber_last_error().decode()


def check(status):
    if status != OK:
        raise AmberError(status, amber_last_error())
    return status


# ------------------------------------------------------------------ same-name wrappers

def amber_abi_version():
    return lib().amber_abi_version()


def amber_column_bytes(desc, col):
    return lib().amber_column_bytes(ctypes.byref(desc), col)


def amber_workspace_bytes(desc):
    return lib().amber_workspace_bytes(ctypes.byref(desc))


def amber_infection_table(beta_num, beta_den, cap=MAX_TABLE):
    """Returns (status, table list, k_sat)."""
    out = (ctypes.c_uint32 * cap)()
    k_sat = ctypes.c_uint32(0)
    st = lib().amber_infection_table(beta_num, beta_den, out, cap, ctypes.byref(k_sat))
    if st != OK:
        return st, None, None
    return st, list(out[:min(cap, k_sat.value + 1)]), k_sat.value


def amber_init_population(desc, bufs, stream_ptr):
    """Returns (status, handle)."""
    h = ctypes.c_void_p()
    st = lib().amber_init_population(ctypes.byref(desc), ctypes.byref(bufs),
                                     ctypes.c_void_p(stream_ptr), ctypes.byref(h))
    return st, h


def amber_init_population_noalloc(desc, bufs, stream_ptr):
    """Returns (status, handle); bufs must carry no workspace."""
    h = ctypes.c_void_p()
    st = lib().amber_init_population_noalloc(ctypes.byref(desc), ctypes.byref(bufs),
                                             ctypes.c_void_p(stream_ptr), ctypes.byref(h))
    return st, h


NOALLOC_SCRATCH_BYTES = 32 << 20


def amber_resume_population(desc, bufs, host_ptrs, step, stream_ptr):
    """Returns (status, handle); host_ptrs[c] is the host address of column c."""
    arr = (ctypes.c_void_p * NUM_COLS)(*host_ptrs)
    h = ctypes.c_void_p()
    st = lib().amber_resume_population(ctypes.byref(desc), ctypes.byref(bufs), arr, step,
                                       ctypes.c_void_p(stream_ptr), ctypes.byref(h))
    return st, h


def amber_view_update(col_ptr, dtype, n, a, b, pred_ptr, pred_dtype, cmp, thr, stream_ptr):
    return lib().amber_view_update(col_ptr, dtype, n, a, b, pred_ptr, pred_dtype, cmp, thr,
                                   stream_ptr)


def amber_view_scatter_workspace_bytes(dtype, n, m):
    return lib().amber_view_scatter_workspace_bytes(dtype, n, m)


def amber_view_scatter_add(col_ptr, dtype, n, ids_ptr, m, vals_ptr, scalar, ws_ptr, ws_bytes,
                           stream_ptr):
    return lib().amber_view_scatter_add(col_ptr, dtype, n, ids_ptr, m, vals_ptr, scalar, ws_ptr,
                                        ws_bytes, stream_ptr)


def amber_step(handle, n_steps):
    return lib().amber_step(handle, n_steps)


def amber_step_batch(handles, n_steps):
    arr = (ctypes.c_void_p * max(1, len(handles)))(*[h.value if isinstance(h, ctypes.c_void_p)
                                                    else h for h in handles])
    return lib().amber_step_batch(arr, len(handles), n_steps)


def amber_read_columns(handle, col_mask, host_ptrs):
    arr = (ctypes.c_void_p * NUM_COLS)(*host_ptrs)
    return lib().amber_read_columns(handle, col_mask, arr)


def amber_invariants(handle):
    """Returns (status, Invariants)."""
    out = Invariants()
    st = lib().amber_invariants(handle, ctypes.byref(out))
    return st, out


def amber_pop_info(handle):
    out = PopInfo()
    st = lib().amber_pop_info(handle, ctypes.byref(out))
    return st, out


def amber_set_tuning(handle, block=256, sir_form=SIR_AUTO, max_groups_per_thread=0,
                     sir_count=COUNT_AUTO, wealth_form=WEALTH_AUTO, sir_tile=0, sir_poll=0):
    t = Tuning(block, sir_form, max_groups_per_thread, sir_count, wealth_form, sir_tile, sir_poll)
    return lib().amber_set_tuning(handle, ctypes.byref(t))


def amber_get_tuning(handle):
    """Returns (status, Tuning)."""
    t = Tuning()
    st = lib().amber_get_tuning(handle, ctypes.byref(t))
    return st, t


def amber_profile_enable(handle, enable):
    return lib().amber_profile_enable(handle, 1 if enable else 0)


def amber_profile_read(handle, cap=32):
    """Returns (status, {kernel name: (launches, total_ms)})."""
    out = (KernelTime * cap)()
    count = ctypes.c_uint32(0)
    st = lib().amber_profile_read(handle, out, cap, ctypes.byref(count))
    if st != OK:
        return st, None
    return st, {out[i].name.decode(): (out[i].launches, out[i].total_ms)
                for i in range(min(cap, count.value))}


def amber_release(handle):
    return lib().amber_release(handle)


# ------------------------------------------------------------------ convenience

def make_desc(model, n, L=0, seed=0, stream=0, wealth_init=1, beta=(1, 20),
              gamma=(1, 100), initial_infected=0):
    return RunDesc(ABI_VERSION, model, n, L, seed & 0xFFFFFFFF, stream & 0xFFFFFFFF,
                   wealth_init, beta[0], beta[1], gamma[0], gamma[1], initial_infected)


def footprint_bytes(desc):
    """Device bytes a run needs: its columns plus its workspace."""
    cols = sum(amber_column_bytes(desc, c) for c in range(NUM_COLS))
    ws = amber_workspace_bytes(desc)
    return cols + ws if ws else 0


_LIVE = weakref.WeakSet()


@atexit.register
def _release_all():
    """Release every live handle while the interpreter, torch and the HIP
    runtime are still whole, rather than from __del__ during teardown."""
    for pop in list(_LIVE):
        try:
            pop.release()
        except Exception:
            pass


class Population:
    """One run: device buffers (torch tensors on the current device) plus the
    library handle.  ``stream`` is a torch.cuda.Stream (default: current).
    ``resume=(host_columns, step)`` continues a run from its state after
    `step` steps (amber_resume_population); ``noalloc`` takes the library's
    device scratch as the workspace (amber_init_population_noalloc)."""

    def __init__(self, model, n, L=0, seed=0, stream_id=0, wealth_init=1, beta=(1, 20),
                 gamma=(1, 100), initial_infected=0, stream=None, device=None,
                 buffers=None, noalloc=False, resume=None):
        import torch
        self.desc = make_desc(model, n, L, seed, stream_id, wealth_init, beta, gamma,
                              initial_infected)
        self.model, self.n = model, n
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        ws = amber_workspace_bytes(self.desc)
        if ws == 0:
            raise AmberError(E_INVALID, amber_last_error())
        self.cols = {}
        b = Buffers()
        for c in MODEL_COLUMNS[model]:
            nb = amber_column_bytes(self.desc, c)
            dtype = torch.uint8 if c == COL_STATE else torch.int32
            t = (buffers or {}).get(c)
            if t is None:
                t = torch.empty(nb // (1 if c == COL_STATE else 4), dtype=dtype, device=dev)
            self.cols[c] = t
            b.col[c] = t.data_ptr()
        if noalloc:
            # the library's device scratch is the workspace
            self.workspace = None
            b.workspace, b.workspace_bytes = None, 0
        else:
            self.workspace = (buffers or {}).get("workspace")
            if self.workspace is None:
                self.workspace = torch.empty(ws, dtype=torch.uint8, device=dev)
            b.workspace = self.workspace.data_ptr()
            b.workspace_bytes = self.workspace.numel()
        self.bufs = b
        self.handle = None
        if resume is not None:
            host_cols, step = resume
            import numpy as np
            self._host = {}
            ptrs = [None] * NUM_COLS
            for c, h in zip(MODEL_COLUMNS[model], host_cols):
                a = np.ascontiguousarray(h, dtype=np.uint8 if c == COL_STATE else np.int32)
                self._host[c] = a
                ptrs[c] = a.ctypes.data
            st, handle = amber_resume_population(self.desc, b, ptrs, step,
                                                 self.stream.cuda_stream)
        else:
            init = amber_init_population_noalloc if noalloc else amber_init_population
            st, handle = init(self.desc, b, self.stream.cuda_stream)
        check(st)
        self.handle = handle
        _LIVE.add(self)

    # --- steps
    def step(self, n_steps=1):
        check(amber_step(self.handle, n_steps))
        return self

    def step_async(self, n_steps=1):
        """Steps under asynchronous (sequential) semantics (amber_step_async);
        the workspace is allocated with torch on first use."""
        import torch
        need = amber_async_workspace_bytes(self.desc)
        ws = getattr(self, "_async_ws", None)
        if ws is None or ws.numel() < need:
            ws = self._async_ws = torch.empty(max(need, 16), dtype=torch.uint8,
                                              device=self.stream.device)
        check(amber_step_async(self.handle, n_steps, ws.data_ptr(), ws.numel()))
        return self

    def info(self):
        st, inf = amber_pop_info(self.handle)
        check(st)
        return inf

    def invariants(self):
        st, inv = amber_invariants(self.handle)
        check(st)
        return inv.as_dict()

    def read(self):
        """Host numpy copies of the model's columns, in column order."""
        import numpy as np
        outs = {}
        ptrs = [None] * NUM_COLS
        mask = 0
        for c in MODEL_COLUMNS[self.model]:
            a = np.empty(self.n, dtype=np.uint8 if c == COL_STATE else np.int32)
            outs[c] = a
            ptrs[c] = a.ctypes.data
            mask |= 1 << c
        check(amber_read_columns(self.handle, mask, ptrs))
        return [outs[c] for c in MODEL_COLUMNS[self.model]]

    def tune(self, block=256, sir_form=SIR_AUTO, max_groups_per_thread=0, sir_count=COUNT_AUTO,
             wealth_form=WEALTH_AUTO, sir_tile=0, sir_poll=0):
        check(amber_set_tuning(self.handle, block, sir_form, max_groups_per_thread, sir_count,
                               wealth_form, sir_tile, sir_poll))
        return self

    def profile(self, enable=True):
        check(amber_profile_enable(self.handle, enable))
        return self

    def kernel_times(self):
        st, t = amber_profile_read(self.handle)
        check(st)
        return t

    def release(self):
        h, self.handle = getattr(self, "handle", None), None
        _LIVE.discard(self)
        if h is not None and h.value:
            check(amber_release(h))

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def amber_view_write_log_workspace_bytes(m):
    return lib().amber_view_write_log_workspace_bytes(m)


def amber_view_write_log(col_ptr, dtype, n, ids_ptr, m, vals_ptr, ws_ptr, ws_bytes, stream_ptr):
    return lib().amber_view_write_log(col_ptr, dtype, n, ids_ptr, m, vals_ptr, ws_ptr, ws_bytes,
                                      stream_ptr)


def amber_async_workspace_bytes(desc):
    return lib().amber_async_workspace_bytes(ctypes.byref(desc))


def amber_step_async(handle, n_steps, ws_ptr, ws_bytes):
    return lib().amber_step_async(handle, n_steps, ws_ptr, ws_bytes)


def write_log(col, ids, vals, stream=None, workspace=None):
    """Buffered writes flushed once into a device tensor, in log order: the
    last write to an id stays; ids outside the column are skipped."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(col.device)
    dt = _dtype_of(col)
    m = ids.numel()
    need = amber_view_write_log_workspace_bytes(m)
    if m and workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=col.device)
    check(amber_view_write_log(col.data_ptr(), dt, col.numel(), ids.data_ptr() if m else None, m,
                               vals.data_ptr() if m else None,
                               workspace.data_ptr() if workspace is not None else None,
                               workspace.numel() if workspace is not None else 0, st.cuda_stream))
    return col


MOORE, VON_NEUMANN = 0, 1


def _dims_arr(dims):
    return (ctypes.c_uint32 * len(dims))(*[int(d) for d in dims])


def _pos_arr(pos):
    return (ctypes.c_void_p * len(pos))(*[p.data_ptr() for p in pos])


def amber_grid_count(pos_ptrs, dims, n, state_ptr, match, counts_ptr, stream_ptr):
    return lib().amber_grid_count((ctypes.c_void_p * len(pos_ptrs))(*pos_ptrs), len(dims),
                                  _dims_arr(dims), n, state_ptr, match, counts_ptr, stream_ptr)


def amber_grid_neighbour_sum(counts_ptr, dims, neighbourhood, torus, out_ptr, stream_ptr):
    return lib().amber_grid_neighbour_sum(counts_ptr, len(dims), _dims_arr(dims), neighbourhood,
                                          torus, out_ptr, stream_ptr)


def amber_grid_gather(table_ptr, pos_ptrs, dims, n, out_ptr, stream_ptr):
    return lib().amber_grid_gather(table_ptr, (ctypes.c_void_p * len(pos_ptrs))(*pos_ptrs),
                                   len(dims), _dims_arr(dims), n, out_ptr, stream_ptr)


def amber_graph_neighbour_count(row_ptr, col_ptr, n, nnz, state_ptr, match, out_ptr, stream_ptr):
    return lib().amber_graph_neighbour_count(row_ptr, col_ptr, n, nnz, state_ptr, match, out_ptr,
                                             stream_ptr)


def amber_sir_transition(state_ptr, k_ptr, n, seed, stream_id, t, t_inf_ptr, table_len, t_rec,
                         stream_ptr):
    return lib().amber_sir_transition(state_ptr, k_ptr, n, seed, stream_id, t, t_inf_ptr,
                                      table_len, t_rec, stream_ptr)


def _cur(dev_tensor, stream):
    import torch
    return (stream if stream is not None else torch.cuda.current_stream(dev_tensor.device)).cuda_stream


def grid_count(dims, pos, state=None, match=1, out=None, stream=None):
    """Agents per cell of an n-D lattice (device tensors; pos = list of int32
    columns), counting those with state == match (all if state is None)."""
    import math
    import torch
    cells = math.prod(int(d) for d in dims)
    out = out if out is not None else torch.empty(cells, dtype=torch.int32, device=pos[0].device)
    check(amber_grid_count([p.data_ptr() for p in pos], dims, pos[0].numel(),
                           state.data_ptr() if state is not None else None, match,
                           out.data_ptr(), _cur(out, stream)))
    return out


def grid_neighbour_sum(dims, counts, neighbourhood=MOORE, torus=True, out=None, stream=None):
    import torch
    out = out if out is not None else torch.empty_like(counts)
    check(amber_grid_neighbour_sum(counts.data_ptr(), dims, neighbourhood, 1 if torus else 0,
                                   out.data_ptr(), _cur(out, stream)))
    return out


def grid_gather(dims, pos, table, out=None, stream=None):
    import torch
    n = pos[0].numel()
    out = out if out is not None else torch.empty(n, dtype=torch.int32, device=table.device)
    check(amber_grid_gather(table.data_ptr(), [p.data_ptr() for p in pos], dims, n,
                            out.data_ptr(), _cur(out, stream)))
    return out


def graph_neighbour_count(row, col, state, match=1, out=None, stream=None):
    import torch
    n = row.numel() - 1
    out = out if out is not None else torch.empty(n, dtype=torch.int32, device=row.device)
    check(amber_graph_neighbour_count(row.data_ptr(), col.data_ptr() if col.numel() else None, n,
                                      col.numel(), state.data_ptr(), match, out.data_ptr(),
                                      _cur(out, stream)))
    return out


def sir_transition(state, k, seed, stream_id, t, beta=(1, 20), gamma=(1, 100), stream=None):
    """The SIR transition of step t in place on a device uint8 state column,
    given each agent's infected count k (device int32/uint32)."""
    import numpy as np
    import torch
    st, table, k_sat = amber_infection_table(*beta)
    check(st)
    t_rec = ctypes.c_uint32(0)
    check(lib().amber_recovery_threshold(gamma[0], gamma[1], ctypes.byref(t_rec)))
    dev_table = torch.from_numpy(np.array(table, dtype=np.uint32).view(np.int32)).to(state.device)
    check(amber_sir_transition(state.data_ptr(), k.data_ptr(), state.numel(), seed, stream_id, t,
                               dev_table.data_ptr(), len(table), t_rec.value, _cur(state, stream)))
    if stream is not None:
        dev_table.record_stream(stream)     # kept until the kernel on `stream` has read it
    return state


class ContRun:
    """The paper's continuous-space walk (sir=False) or SIR in a W x W world,
    on device columns allocated with torch; every step runs in the library's
    kernels (amber_cont_*)."""

    def __init__(self, n, W=100.0, r=5.0, seed=0, stream_id=0, sir=False, p=(1, 10),
                 recover=14, initial_infected=5, stream=None):
        import torch
        self.n, self.W, self.r, self.seed, self.stream_id = n, float(W), float(r), seed, stream_id
        self.sir, self.p, self.recover, self.t = sir, p, recover, 0
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        dev = self.stream.device
        self.x = torch.empty(n, dtype=torch.float32, device=dev)
        self.y = torch.empty(n, dtype=torch.float32, device=dev)
        self.s = self.days = self.ws = None
        if sir:
            self.s = torch.empty(n, dtype=torch.uint8, device=dev)
            self.days = torch.empty(n, dtype=torch.uint8, device=dev)
            need = lib().amber_cont_sir_workspace_bytes(n, self.W, self.r, p[0], p[1])
            if need == 0:
                raise AmberError(E_INVALID, "continuous SIR arguments refused")
            self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        ptr = lambda t: t.data_ptr() if t is not None else None
        check(lib().amber_cont_init(self.x.data_ptr(), self.y.data_ptr(), ptr(self.s),
                                    ptr(self.days), n, self.W, seed, stream_id,
                                    initial_infected if sir else 0, self.stream.cuda_stream))

    def step(self, k=1):
        if self.sir:
            check(lib().amber_cont_sir(self.x.data_ptr(), self.y.data_ptr(), self.s.data_ptr(),
                                       self.days.data_ptr(), self.n, self.W, self.r, self.seed,
                                       self.stream_id, self.p[0], self.p[1], self.recover, self.t,
                                       k, self.ws.data_ptr(), self.ws.numel(),
                                       self.stream.cuda_stream))
        else:
            check(lib().amber_cont_walk(self.x.data_ptr(), self.y.data_ptr(), self.n, self.W,
                                        self.seed, self.stream_id, self.t, k,
                                        self.stream.cuda_stream))
        self.t += k
        return self

    def read(self):
        self.stream.synchronize()
        cols = [self.x, self.y] + ([self.s, self.days] if self.sir else [])
        return [c.cpu().numpy() for c in cols]


def _dtype_of(t):
    import torch
    if t.dtype == torch.int32:
        return DT_I32
    if t.dtype == torch.float32:
        return DT_F32
    raise TypeError("view columns must be int32 or float32 tensors")


def view_update(col, a, b, pred=None, cmp="<", thr=0, stream=None):
    """Full (pred None) or filtered view update of a device tensor in place:
    col[r] = a*col[r] + b where pred[r] CMP thr (pred read before the update)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(col.device)
    dt = _dtype_of(col)
    pdt = _dtype_of(pred) if pred is not None else DT_I32
    check(amber_view_update(col.data_ptr(), dt, col.numel(), value(dt, a), value(dt, b),
                            pred.data_ptr() if pred is not None else None, pdt, CMP[cmp],
                            value(pdt, thr), st.cuda_stream))
    return col


def scatter_add(col, ids, vals=None, scalar=0, stream=None, workspace=None):
    """Scatter view on a device tensor in place: col[ids[j]] += vals[j] (or
    scalar) in list order, duplicates accumulating; ids a uint32-valued
    int32 tensor on the device.  A float32 scatter needs a workspace; one is
    allocated with torch when none is passed."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(col.device)
    dt = _dtype_of(col)
    m = ids.numel()
    need = amber_view_scatter_workspace_bytes(dt, col.numel(), m)
    if need and workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=col.device)
    check(amber_view_scatter_add(col.data_ptr(), dt, col.numel(), ids.data_ptr() if m else None,
                                 m, vals.data_ptr() if vals is not None else None,
                                 value(dt, scalar),
                                 workspace.data_ptr() if workspace is not None else None,
                                 workspace.numel() if workspace is not None else 0,
                                 st.cuda_stream))
    return col


def step_batch(pops, n_steps):
    check(amber_step_batch([p.handle for p in pops], n_steps))
