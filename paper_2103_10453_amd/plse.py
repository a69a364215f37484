"""Python binding of libplse (include/plse.h): argument marshalling only.

Every computation runs in the HIP kernels of libplse.so; PyTorch supplies the
device workspace and the stream.  There is no CPU fallback: if libplse.so is
missing or cannot be loaded, every call raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplse.so")

PLSE_OK, PLSE_E_ARG, PLSE_E_GRID, PLSE_E_WORKSPACE, PLSE_E_HIP, PLSE_E_BUSY, PLSE_PENDING, \
    PLSE_E_PARAM, PLSE_E_CAPACITY, PLSE_E_FAULT, PLSE_E_CANCELLED = range(11)
NCOUNTERS = 9
COUNTER_NAMES = ["iters", "moves", "idle", "cands", "elig", "nupd", "snaps", "repairs", "cupd"]
HIST = 64
MAX_GENERATIONS = 65536


class PlseError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib().plse_strerror(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("generations_run", ctypes.c_int32), ("best_f", ctypes.c_int32),
                ("best_generation", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
                ("totals", ctypes.c_uint64 * NCOUNTERS)]


class Progress(ctypes.Structure):
    _fields_ = [("generations_run", ctypes.c_int32), ("best_f", ctypes.c_int32),
                ("best_generation", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
                ("iterations", ctypes.c_uint64)]


class Timing(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("best_s", ctypes.c_double),
                ("generations", ctypes.c_int32), ("best_generation", ctypes.c_int32),
                ("filled", ctypes.c_int32), ("status", ctypes.c_int32),
                ("moves", ctypes.c_uint64)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        # torch's HIP runtime first: the library then binds to that same
        # runtime (by soname) instead of loading a second one beside it
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                ctypes.c_size_t)
        sigs = {
            "plse_create": [i32, P, P],
            "plse_info": [P, P, P, P],
            "plse_row_stride": [P, P],
            "plse_sizes": [P, P, P, P, P],
            "plse_set_param": [P, ctypes.c_char_p, i64],
            "plse_get_param": [P, ctypes.c_char_p, P],
            "plse_workspace_bytes": [P, i32, P],
            "plse_attach_workspace": [P, P, sz],
            "plse_solve": [P, i32, i32, u64, P, P, P],
            "plse_begin": [P, i32, u64, P],
            "plse_solve_batch": [P, i32, i32, i32, P, P, P, P],
            "plse_batch_begin": [P, i32, i32, P, P, P],
            "plse_batch_step": [P, i32, P],
            "plse_batch_end": [P, P, P, P],
            "plse_solve_noalloc": [P, i32, i32, u64, P, P, P, P],
            "plse_measure_lds_bandwidth": [P, i32, P],
            "plse_step": [P, i32, P],
            "plse_end": [P, P, P, P],
            "plse_peek": [P, P, P],
            "plse_autotune": [P, i32, i32, u64, P, P],
            "plse_autotune_shape": [P, i32, i32, u64, P, P],
            "plse_checkpoint": [P, P, P, sz, P],
            "plse_resume": [P, i32, P, P, sz],
            "plse_last_timing": [P, P, P, P],
            "plse_last_stage_timing": [P, P, P],
            "plse_last_stats": [P, P, P, P],
            "plse_stage_init": [P, i32, u64, P, P, P],
            "plse_stage_plits": [P, i32, i32, u64, P, P, P, P, P],
            "plse_stage_distances": [P, i32, P, P, P],
            "plse_stage_select": [P, i32, i32, u64, P, P, P, P],
            "plse_stage_match": [P, i32, P, P, P, P, P, P, P],
            "plse_stage_aux": [P, i32, i32, u64, P, P, P, P, P],
            "plse_server_create": [sz, P, i32, P, P],
            "plse_server_submit": [P, P, i32, i32, u64, P],
            "plse_server_poll": [P, u64, P, P, P],
            "plse_server_status": [P, P, P, P],
            "plse_server_cancel": [P, u64],
            "plse_server_destroy": [P],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.plse_destroy.argtypes = [P]
        L.plse_destroy.restype = None
        L.plse_strerror.argtypes = [ctypes.c_int]
        L.plse_strerror.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def library_path() -> str:
    return LIB_PATH


def exported_symbols():
    """Names of the C-ABI functions the binding resolves."""
    L = _lib()
    names = ["plse_create", "plse_info", "plse_sizes", "plse_row_stride", "plse_set_param", "plse_get_param",
             "plse_workspace_bytes", "plse_attach_workspace", "plse_solve", "plse_solve_batch",
             "plse_solve_noalloc", "plse_batch_begin", "plse_batch_step", "plse_batch_end", "plse_measure_lds_bandwidth",
             "plse_begin",
             "plse_step", "plse_end", "plse_peek", "plse_autotune", "plse_autotune_shape", "plse_checkpoint", "plse_resume", "plse_last_timing", "plse_last_stage_timing", "plse_last_stats",
             "plse_destroy", "plse_strerror", "plse_stage_init", "plse_stage_plits",
             "plse_stage_distances", "plse_stage_select", "plse_stage_match", "plse_stage_aux",
             "plse_server_create", "plse_server_submit", "plse_server_poll", "plse_server_status",
             "plse_server_cancel",
             "plse_server_destroy"]
    return [n for n in names if hasattr(L, n)]


def _check(status: int, where: str):
    if status != PLSE_OK:
        raise PlseError(status, where)


def _np(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# --- the C calls, same names --------------------------------------------------------
def plse_create(grid) -> ctypes.c_void_p:
    g = np.ascontiguousarray(np.asarray(grid, dtype=np.int8))
    n = g.shape[0]
    if g.shape != (n, n):
        raise ValueError("grid must be n x n")
    h = ctypes.c_void_p()
    _check(_lib().plse_create(n, _np(g), ctypes.byref(h)), "plse_create")
    return h


def plse_info(h):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib().plse_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "plse_info")
    return a.value, b.value, c.value


def plse_sizes(h):
    a, b, c, d = (ctypes.c_int32() for _ in range(4))
    _check(_lib().plse_sizes(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)),
           "plse_sizes")
    return a.value, b.value, c.value, d.value


def plse_row_stride(h) -> int:
    s = ctypes.c_int32()
    _check(_lib().plse_row_stride(h, ctypes.byref(s)), "plse_row_stride")
    return s.value


def plse_set_param(h, key: str, value: int):
    _check(_lib().plse_set_param(h, key.encode(), int(value)), f"plse_set_param({key})")


def plse_get_param(h, key: str) -> int:
    v = ctypes.c_int64()
    _check(_lib().plse_get_param(h, key.encode(), ctypes.byref(v)), f"plse_get_param({key})")
    return v.value


def plse_workspace_bytes(h, population: int) -> int:
    b = ctypes.c_size_t()
    _check(_lib().plse_workspace_bytes(h, population, ctypes.byref(b)), "plse_workspace_bytes")
    return b.value


def plse_attach_workspace(h, tensor):
    if tensor is None:
        _check(_lib().plse_attach_workspace(h, None, 0), "plse_attach_workspace")
    else:
        _check(_lib().plse_attach_workspace(h, _dev(tensor), tensor.numel() * tensor.element_size()),
               "plse_attach_workspace")


def plse_solve(h, n: int, population: int, generations: int, seed: int, stream=None):
    grid = np.zeros((n, n), dtype=np.int8)
    filled = ctypes.c_int32()
    _check(_lib().plse_solve(h, population, generations, seed & ((1 << 64) - 1), _stream(stream),
                             _np(grid), ctypes.byref(filled)), "plse_solve")
    return grid, filled.value


NOALLOC_BYTES = 64 << 20  # PLSE_NOALLOC_BYTES


def plse_solve_noalloc(h, n: int, population: int, generations: int, seed: int, stream=None):
    """plse_solve on the library's fixed device array (no workspace, no
    allocation); returns (grid, filled, bytes_needed)."""
    grid = np.zeros((n, n), dtype=np.int8)
    filled = ctypes.c_int32()
    need = ctypes.c_size_t()
    _check(_lib().plse_solve_noalloc(h, population, generations, seed & ((1 << 64) - 1),
                                     _stream(stream), _np(grid), ctypes.byref(filled),
                                     ctypes.byref(need)), "plse_solve_noalloc")
    return grid, filled.value, need.value


def plse_measure_lds_bandwidth(repeats: int = 5, stream=None) -> float:
    """Sustained LDS read bandwidth of the current GPU, bytes/s."""
    bw = ctypes.c_double()
    _check(_lib().plse_measure_lds_bandwidth(_stream(stream), repeats, ctypes.byref(bw)),
           "plse_measure_lds_bandwidth")
    return bw.value


def plse_solve_batch(handles, ns, population: int, generations: int, seeds, stream=None):
    """Solve several instances in one batched run; returns [(grid, filled)]."""
    count = len(handles)
    hs = (ctypes.c_void_p * count)(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                     for h in handles])
    sd = (ctypes.c_uint64 * count)(*[s & ((1 << 64) - 1) for s in seeds])
    grids = [np.zeros((n, n), dtype=np.int8) for n in ns]
    gp = (ctypes.c_void_p * count)(*[g.ctypes.data for g in grids])
    filled = np.zeros(count, dtype=np.int32)
    _check(_lib().plse_solve_batch(hs, count, population, generations, sd, _stream(stream), gp,
                                   _np(filled)), "plse_solve_batch")
    return [(grids[i], int(filled[i])) for i in range(count)]


def plse_batch_begin(handles, population: int, seeds, stream=None):
    count = len(handles)
    hs = (ctypes.c_void_p * count)(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                     for h in handles])
    sd = (ctypes.c_uint64 * count)(*[s & ((1 << 64) - 1) for s in seeds])
    b = ctypes.c_void_p()
    _check(_lib().plse_batch_begin(hs, count, population, sd, _stream(stream), ctypes.byref(b)),
           "plse_batch_begin")
    return b


def plse_batch_step(b, generations: int, stream=None):
    _check(_lib().plse_batch_step(b, generations, _stream(stream)), "plse_batch_step")


def plse_batch_end(b, ns, stream=None):
    grids = [np.zeros((n, n), dtype=np.int8) for n in ns]
    gp = (ctypes.c_void_p * len(ns))(*[g.ctypes.data for g in grids])
    filled = np.zeros(len(ns), dtype=np.int32)
    _check(_lib().plse_batch_end(b, _stream(stream), gp, _np(filled)), "plse_batch_end")
    return [(grids[i], int(filled[i])) for i in range(len(ns))]


def plse_begin(h, population: int, seed: int, stream=None):
    _check(_lib().plse_begin(h, population, seed & ((1 << 64) - 1), _stream(stream)), "plse_begin")


def plse_step(h, generations: int, stream=None):
    _check(_lib().plse_step(h, generations, _stream(stream)), "plse_step")


def plse_end(h, n: int, stream=None):
    grid = np.zeros((n, n), dtype=np.int8)
    filled = ctypes.c_int32()
    _check(_lib().plse_end(h, _stream(stream), _np(grid), ctypes.byref(filled)), "plse_end")
    return grid, filled.value


def plse_peek(h, stream=None):
    pr = Progress()
    _check(_lib().plse_peek(h, _stream(stream), ctypes.byref(pr)), "plse_peek")
    return dict(generations_run=pr.generations_run, best_f=pr.best_f,
                best_generation=pr.best_generation, stop_reason=pr.stop_reason,
                iterations=int(pr.iterations))


def plse_autotune(h, sample: int, depth: int, seed: int, stream=None):
    ms = np.zeros(3, dtype=np.float32)
    _check(_lib().plse_autotune(h, sample, depth, seed & ((1 << 64) - 1), _stream(stream),
                                _np(ms)), "plse_autotune")
    return ms


def plse_autotune_shape(h, sample: int, depth: int, seed: int, stream=None):
    ms = np.zeros(9, dtype=np.float32)
    _check(_lib().plse_autotune_shape(h, sample, depth, seed & ((1 << 64) - 1), _stream(stream),
                                      _np(ms)), "plse_autotune_shape")
    return ms.reshape(3, 3)


def plse_checkpoint(h, stream=None) -> np.ndarray:
    n = ctypes.c_size_t()
    _check(_lib().plse_checkpoint(h, _stream(stream), None, 0, ctypes.byref(n)), "plse_checkpoint")
    buf = np.zeros(n.value, dtype=np.uint8)
    _check(_lib().plse_checkpoint(h, _stream(stream), _np(buf), buf.nbytes, ctypes.byref(n)),
           "plse_checkpoint")
    return buf


def plse_resume(h, population: int, image, stream=None):
    image = np.ascontiguousarray(np.asarray(image, dtype=np.uint8))
    _check(_lib().plse_resume(h, population, _stream(stream), _np(image), image.nbytes),
           "plse_resume")


def plse_last_timing(h):
    k = ctypes.c_int32()
    _check(_lib().plse_last_timing(h, ctypes.byref(k), None, None), "plse_last_timing")
    a = np.zeros(max(k.value, 1), dtype=np.float32)
    b = np.zeros(max(k.value, 1), dtype=np.float32)
    _check(_lib().plse_last_timing(h, ctypes.byref(k), _np(a), _np(b)), "plse_last_timing")
    return a[:k.value], b[:k.value]


STAGES = ["distances_Pt", "tabu_search", "best", "distances_new", "selection", "matching",
          "crossover"]


def plse_last_stage_timing(h):
    """Per-stage ms of the last stage-timed session: array [generations, 7]."""
    k = ctypes.c_int32()
    _check(_lib().plse_last_stage_timing(h, ctypes.byref(k), None), "plse_last_stage_timing")
    a = np.zeros((max(k.value, 1), len(STAGES)), dtype=np.float32)
    _check(_lib().plse_last_stage_timing(h, ctypes.byref(k), _np(a)), "plse_last_stage_timing")
    return a[:k.value]


def plse_last_stats(h):
    st = Stats()
    _check(_lib().plse_last_stats(h, ctypes.byref(st), None, None), "plse_last_stats")
    g = st.generations_run
    bf = np.zeros(max(g, 1), dtype=np.int32)
    cnt = np.zeros((max(g, 1), NCOUNTERS), dtype=np.uint64)
    _check(_lib().plse_last_stats(h, ctypes.byref(st), _np(bf), _np(cnt)), "plse_last_stats")
    return dict(generations_run=g, best_f=st.best_f, best_generation=st.best_generation,
                stop_reason=st.stop_reason, totals=np.array(st.totals[:], dtype=np.uint64), best_f_per_gen=bf[:g],
                counters_per_gen=cnt[:g])


def plse_destroy(h):
    if h:
        _lib().plse_destroy(h)


def plse_stage_init(h, population, seed, S, f, stream=None):
    _check(_lib().plse_stage_init(h, population, seed, _stream(stream), _dev(S), _dev(f)),
           "plse_stage_init")


def plse_stage_plits(h, population, gen, seed, S_in, S_out, f_out, counters, stream=None):
    _check(_lib().plse_stage_plits(h, population, gen, seed, _stream(stream), _dev(S_in),
                                   _dev(S_out), _dev(f_out), _dev(counters)), "plse_stage_plits")


def plse_stage_distances(h, m, S, D, stream=None):
    _check(_lib().plse_stage_distances(h, m, _stream(stream), _dev(S), _dev(D)),
           "plse_stage_distances")


def plse_stage_select(h, population, gen, seed, f_all, D_all, accepted, stream=None):
    _check(_lib().plse_stage_select(h, population, gen, seed, _stream(stream), _dev(f_all),
                                    _dev(D_all), _dev(accepted)), "plse_stage_select")


def plse_stage_match(h, population, D, uid, hist, hcount, partner, dpart, stream=None):
    _check(_lib().plse_stage_match(h, population, _stream(stream), _dev(D), _dev(uid), _dev(hist),
                                   _dev(hcount), _dev(partner), _dev(dpart)), "plse_stage_match")


def plse_stage_aux(h, population, gen, seed, S, partner, dpart, S_off, stream=None):
    _check(_lib().plse_stage_aux(h, population, gen, seed, _stream(stream), _dev(S), _dev(partner),
                                 _dev(dpart), _dev(S_off)), "plse_stage_aux")


# --- convenience wrapper -------------------------------------------------------------
class Solver:
    """One instance: handle + a torch-owned device workspace."""

    def __init__(self, grid, device="cuda", **params):
        self.grid = np.ascontiguousarray(np.asarray(grid, dtype=np.int8))
        self.n = self.grid.shape[0]
        self.h = plse_create(self.grid)
        self.nv, self.l, self.ub = plse_info(self.h)
        self.stride = plse_row_stride(self.h)
        self.nd = plse_sizes(self.h)[2]
        self.device = device
        self._ws = None
        self._ws_pop = 0
        for k, v in params.items():
            plse_set_param(self.h, k, v)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            # at interpreter shutdown the module globals may already be gone
            try:
                plse_attach_workspace(h, None)
            except Exception:
                pass
            try:
                plse_destroy(h)
            except Exception:
                pass

    def set_param(self, key, value):
        plse_set_param(self.h, key, value)

    def get_param(self, key):
        return plse_get_param(self.h, key)

    def ensure_workspace(self, population: int):
        import torch
        need = plse_workspace_bytes(self.h, population)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            plse_attach_workspace(self.h, self._ws)
        self._ws_pop = max(self._ws_pop, population)
        return self._ws

    def solve(self, population: int, generations: int, seed: int, stream=None):
        self.ensure_workspace(population)
        return plse_solve(self.h, self.n, population, generations, seed, stream)

    def begin(self, population: int, seed: int, stream=None):
        self.ensure_workspace(population)
        plse_begin(self.h, population, seed, stream)

    def step(self, generations: int, stream=None):
        plse_step(self.h, generations, stream)

    def end(self, stream=None):
        return plse_end(self.h, self.n, stream)

    def peek(self, stream=None):
        return plse_peek(self.h, stream)

    def checkpoint(self, stream=None):
        """Image (uint8 array) of the open session at its generation boundary."""
        return plse_checkpoint(self.h, stream)

    def resume(self, population: int, image, stream=None):
        """Open a session from a checkpoint image (instead of begin)."""
        self.ensure_workspace(population)
        plse_resume(self.h, population, image, stream)

    def autotune(self, sample: int = 4096, depth: int = 2000, seed: int = 1, stream=None):
        """Measure the chunk sizes on `sample` individuals and keep the
        fastest; returns the times (ms) for slots per lane 2, 4, 8 (-1: does
        not fit)."""
        self.ensure_workspace(sample)
        return plse_autotune(self.h, sample, depth, seed, stream)

    def autotune_shape(self, sample: int = 4096, depth: int = 2000, seed: int = 1, stream=None):
        """Measure chunk size x waves per block and keep the fastest; returns
        the times (ms) as [waves 1, 2, 4][slots 2, 4, 8] (-1: does not fit)."""
        self.ensure_workspace(sample)
        return plse_autotune_shape(self.h, sample, depth, seed, stream)

    def timing(self):
        return plse_last_timing(self.h)

    def stats(self):
        return plse_last_stats(self.h)

    def stage_timing(self):
        return plse_last_stage_timing(self.h)

    @staticmethod
    def solve_batch(solvers, population: int, generations: int, seeds, stream=None):
        """Batched plse_solve over several Solver objects (one workspace each)."""
        for s in solvers:
            s.ensure_workspace(population)
        return plse_solve_batch([s.h for s in solvers], [s.n for s in solvers], population,
                                generations, seeds, stream)

    # stage helpers returning torch tensors
    def new_pop(self, count: int):
        import torch
        return torch.zeros((count, self.stride), dtype=torch.uint8, device=self.device)

    def stage_init(self, population: int, seed: int):
        import torch
        self.ensure_workspace(population)
        S = self.new_pop(population)
        f = torch.zeros(population, dtype=torch.int32, device=self.device)
        plse_stage_init(self.h, population, seed, S, f)
        return S, f

    def stage_plits(self, S_in, gen: int, seed: int):
        import torch
        p = S_in.shape[0]
        self.ensure_workspace(p)
        S_out = self.new_pop(p)
        f = torch.zeros(p, dtype=torch.int32, device=self.device)
        cnt = torch.zeros((p, NCOUNTERS), dtype=torch.int64, device=self.device)
        plse_stage_plits(self.h, p, gen, seed, S_in, S_out, f, cnt)
        return S_out, f, cnt

    def stage_distances(self, S):
        import torch
        m = S.shape[0]
        self.ensure_workspace(max(2, (m + 1) // 2))
        D = torch.zeros((m, m), dtype=torch.int16, device=self.device)
        plse_stage_distances(self.h, m, S, D)
        return D

    def stage_select(self, f_all, D_all, gen: int, seed: int):
        import torch
        p = f_all.shape[0] // 2
        self.ensure_workspace(p)
        acc = torch.zeros(p, dtype=torch.int32, device=self.device)
        plse_stage_select(self.h, p, gen, seed, f_all, D_all, acc)
        return acc

    def stage_match(self, D, uid, hist, hcount):
        import torch
        p = D.shape[0]
        self.ensure_workspace(p)
        partner = torch.zeros(p, dtype=torch.int32, device=self.device)
        dpart = torch.zeros(p, dtype=torch.int32, device=self.device)
        plse_stage_match(self.h, p, D, uid, hist, hcount, partner, dpart)
        return partner, dpart

    def stage_aux(self, S, partner, dpart, gen: int, seed: int):
        p = S.shape[0]
        self.ensure_workspace(p)
        S_off = self.new_pop(p)
        plse_stage_aux(self.h, p, gen, seed, S, partner, dpart, S_off)
        return S_off


# --- serving ---------------------------------------------------------------------------
def plse_server_create(budget_bytes: int, arena, max_slots: int, stream):
    srv = ctypes.c_void_p()
    _check(_lib().plse_server_create(budget_bytes, _dev(arena), max_slots, _stream(stream),
                                     ctypes.byref(srv)), "plse_server_create")
    return srv


def plse_server_submit(srv, h, population: int, generations: int, seed: int) -> int:
    t = ctypes.c_uint64()
    _check(_lib().plse_server_submit(srv, h, population, generations, seed & ((1 << 64) - 1),
                                     ctypes.byref(t)), "plse_server_submit")
    return t.value


def plse_server_poll(srv, ticket: int, n: int):
    """None while pending, else (status, grid, filled, Timing)."""
    grid = np.zeros((n, n), dtype=np.int8)
    filled = ctypes.c_int32()
    t = Timing()
    st = _lib().plse_server_poll(srv, ticket, _np(grid), ctypes.byref(filled), ctypes.byref(t))
    if st == PLSE_PENDING:
        return None
    if st == PLSE_E_ARG:
        raise PlseError(st, "plse_server_poll")
    return st, grid, filled.value, t


def plse_server_cancel(srv, ticket: int):
    _check(_lib().plse_server_cancel(srv, ticket), "plse_server_cancel")


def plse_server_status(srv):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib().plse_server_status(srv, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "plse_server_status")
    return a.value, b.value, c.value


def plse_server_destroy(srv):
    if srv:
        _lib().plse_server_destroy(srv)


class Server:
    """Continuous-batching server on a torch-owned device arena."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, device="cuda"):
        import torch
        self.arena = torch.empty(budget_bytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.Stream(device=device)
        self.srv = plse_server_create(budget_bytes, self.arena, max_slots, self.stream)
        self.live = {}

    def submit(self, solver, population: int, generations: int, seed: int) -> int:
        t = plse_server_submit(self.srv, solver.h, population, generations, seed)
        self.live[t] = solver
        return t

    def poll(self, ticket: int):
        solver = self.live[ticket]
        r = plse_server_poll(self.srv, ticket, solver.n)
        if r is None:
            return None
        del self.live[ticket]
        st, grid, filled, t = r
        return dict(status=st, grid=grid, filled=filled, submit_s=t.submit_s, admit_s=t.admit_s,
                    done_s=t.done_s, best_s=t.best_s, generations=t.generations,
                    best_generation=t.best_generation, moves=int(t.moves))

    def status(self):
        return plse_server_status(self.srv)

    def cancel(self, ticket: int):
        plse_server_cancel(self.srv, ticket)

    def close(self):
        if self.srv:
            plse_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
