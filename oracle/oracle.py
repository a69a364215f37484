"""ctypes wrapper of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

NPARAMS = 14
P_DEPTH1, P_DEPTH2, P_ALPHA_NUM, P_ALPHA_DEN, P_BETA_NUM, P_BETA_DEN, P_SPACING, \
    P_STOP_AT_UB, P_HIST, P_PARANOID, P_CROSSOVER, P_MATCHING, P_VARIANT, \
    P_MAX_ITERS = range(NPARAMS)
X_AUX, X_UX, X_NONE = 0, 1, 2        # crossover variants (Section 3.5.2, Section 5.2)
M_NEAREST, M_RANDOM = 0, 1           # matching variants (Section 3.5.1, Section 5.3)
V_MPMA, V_PARTIAL = 0, 1             # MPMA, Partial-MPMA (Section 3.7)

NCOUNTERS = 9
COUNTER_NAMES = ["iters", "moves", "idle", "cands", "elig", "nupd", "snaps", "repairs", "cupd"]
HMAX = 64


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O3, OpenMP over individuals)."""
    src = os.path.join(HERE, "mpma_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", LIB_PATH + ".tmp", src]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, u32, u64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        L.orc_create.restype = P
        L.orc_create.argtypes = [i32, P, P]
        L.orc_destroy.argtypes = [P]
        L.orc_info.argtypes = [P, P]
        L.orc_tables.argtypes = [P, P, P, P, P]
        L.orc_philox.argtypes = [P, P, P]
        L.orc_fmix32.restype = u32
        L.orc_fmix32.argtypes = [u32]
        L.orc_tie16.restype = u32
        L.orc_tie16.argtypes = [u32, u32, u32, u32]
        L.orc_init.argtypes = [P, u64, i32, P, P]
        L.orc_init_slots.argtypes = [P, u64, i32, P, P, P]
        L.orc_plits.argtypes = [P, P, u64, i32, i32, P, P, P, P, P]
        L.orc_plits_trace.restype = i32
        L.orc_plits_trace.argtypes = [P, P, u64, i32, i32, P, i32, P]
        L.orc_distances.argtypes = [i32, i32, P, i32, P, P]
        L.orc_select.argtypes = [i32, i32, ctypes.c_int64, u64, i32, P, P, P]
        L.orc_match.argtypes = [i32, P, P, P, P, i32, P, P]
        L.orc_match_mode.argtypes = [i32, P, P, P, P, i32, i32, u64, i32, P, P]
        L.orc_aux.argtypes = [i32, i32, u64, i32, ctypes.c_int64, ctypes.c_int64, P, P, P, P]
        L.orc_aux_mode.argtypes = [i32, i32, u64, i32, ctypes.c_int64, ctypes.c_int64, i32, P,
                                   P, P, P]
        L.orc_run.restype = i32
        L.orc_run.argtypes = [P, P, i32, i32, u64, P, P, P, P, P, P]
        L.orc_run_state.restype = i32
        L.orc_run_state.argtypes = [P, P, i32, i32, u64, P, P, P, P, P, P, P]
        L.orc_aux_threshold.restype = u64
        L.orc_aux_threshold.argtypes = [ctypes.c_int64, ctypes.c_int64, i32, i32]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_params(nv: int, n: int, depth: int | None = None, stop_at_ub: bool = False,
                   paranoid: bool = False, crossover: int = X_AUX,
                   matching: int = M_NEAREST, variant: int = V_MPMA,
                   max_iterations: int = 0) -> np.ndarray:
    """Paper defaults (Table 1, Section 3.3) with an optional total depth.

    With a depth d, phase 2 keeps its 2|V| iterations and phase 1 gets the rest.
    """
    P = np.zeros(NPARAMS, dtype=np.int64)
    if depth is None:
        P[P_DEPTH1], P[P_DEPTH2] = 100 * nv, 2 * nv
    else:
        d2 = min(2 * nv, depth)
        P[P_DEPTH1], P[P_DEPTH2] = depth - d2, d2
    P[P_ALPHA_NUM], P[P_ALPHA_DEN] = 6, 10
    P[P_BETA_NUM], P[P_BETA_DEN] = 20, 1
    P[P_SPACING] = 10
    P[P_STOP_AT_UB] = int(stop_at_ub)
    P[P_HIST] = 64
    P[P_PARANOID] = int(paranoid)
    P[P_CROSSOVER] = int(crossover)
    P[P_MATCHING] = int(matching)
    P[P_VARIANT] = int(variant)
    P[P_MAX_ITERS] = int(max_iterations)
    return P


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def fmix32(x: int) -> int:
    return int(lib().orc_fmix32(x & 0xFFFFFFFF))


def tie16(wv: int, wk: int, v: int, k: int) -> int:
    return int(lib().orc_tie16(wv & 0xFFFFFFFF, wk & 0xFFFFFFFF, v, k))


class Instance:
    """Reduced Latin square graph of one grid (Alg. 1)."""

    def __init__(self, grid):
        g = np.ascontiguousarray(np.asarray(grid, dtype=np.int8))
        self.n = int(g.shape[0])
        self.grid = g
        st = np.zeros(1, dtype=np.int32)
        self.h = lib().orc_create(self.n, _ptr(g), _ptr(st))
        self.status = int(st[0])
        if not self.h:
            raise ValueError(f"invalid grid (status {self.status})")
        info = np.zeros(4, dtype=np.int32)
        lib().orc_info(self.h, _ptr(info))
        self.nv, self.l, self.ub, self.nd = (int(x) for x in info)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self.h = None

    def tables(self):
        vr = np.zeros(self.nv, dtype=np.int32)
        vc = np.zeros(self.nv, dtype=np.int32)
        off = np.zeros(self.nv + 1, dtype=np.int32)
        dom = np.zeros(max(self.nd, 1), dtype=np.uint8)
        lib().orc_tables(self.h, _ptr(vr), _ptr(vc), _ptr(off), _ptr(dom))
        return vr, vc, off, dom[: self.nd]

    def params(self, depth=None, **kw):
        return default_params(self.nv, self.n, depth=depth, **kw)

    def init(self, seed: int, p: int):
        S = np.zeros((p, self.nv), dtype=np.uint8)
        f = np.zeros(p, dtype=np.int32)
        lib().orc_init(self.h, seed, p, _ptr(S), _ptr(f))
        return S, f

    def init_slots(self, seed: int, slots):
        slots = np.ascontiguousarray(np.asarray(slots, dtype=np.int32))
        S = np.zeros((len(slots), self.nv), dtype=np.uint8)
        f = np.zeros(len(slots), dtype=np.int32)
        lib().orc_init_slots(self.h, seed, len(slots), _ptr(slots), _ptr(S), _ptr(f))
        return S, f

    def plits(self, params, seed: int, gen: int, slots, S_in):
        slots = np.ascontiguousarray(np.asarray(slots, dtype=np.int32))
        S_in = np.ascontiguousarray(np.asarray(S_in, dtype=np.uint8)).reshape(len(slots), self.nv)
        S_out = np.zeros_like(S_in)
        f = np.zeros(len(slots), dtype=np.int32)
        cnt = np.zeros((len(slots), NCOUNTERS), dtype=np.uint64)
        P = np.ascontiguousarray(params, dtype=np.int64)
        lib().orc_plits(self.h, _ptr(P), seed, gen, len(slots), _ptr(slots), _ptr(S_in),
                        _ptr(S_out), _ptr(f), _ptr(cnt))
        return S_out, f, cnt

    def plits_trace(self, params, seed: int, gen: int, slot: int, S_in, max_rows: int = 100000):
        rows = np.zeros((max_rows, 7), dtype=np.int64)
        S_in = np.ascontiguousarray(np.asarray(S_in, dtype=np.uint8))
        P = np.ascontiguousarray(params, dtype=np.int64)
        k = lib().orc_plits_trace(self.h, _ptr(P), seed, gen, slot, _ptr(S_in), max_rows,
                                  _ptr(rows))
        return rows[:k]

    def run(self, params, p: int, G: int, seed: int):
        grid = np.zeros((self.n, self.n), dtype=np.int8)
        filled = np.zeros(1, dtype=np.int32)
        bf = np.zeros(G, dtype=np.int32)
        cnt = np.zeros((G, NCOUNTERS), dtype=np.uint64)
        fS = np.zeros((p, self.nv), dtype=np.uint8)
        ff = np.zeros(p, dtype=np.int32)
        P = np.ascontiguousarray(params, dtype=np.int64)
        gens = lib().orc_run(self.h, _ptr(P), p, G, seed, _ptr(grid), _ptr(filled), _ptr(bf),
                             _ptr(cnt), _ptr(fS), _ptr(ff))
        if gens < 0:
            raise ValueError("bad run arguments")
        return dict(grid=grid, filled=int(filled[0]), best_f=bf, counters=cnt, gens=int(gens),
                    final_S=fS, final_f=ff)

    def run_state(self, params, p: int, G: int, seed: int):
        """run() plus the state of Alg. 2 at the end: uids, partner histories
        (ring of HMAX per individual) and their counts, the offspring waiting
        for the next search, and S*."""
        grid = np.zeros((self.n, self.n), dtype=np.int8)
        filled = np.zeros(1, dtype=np.int32)
        bf = np.zeros(G, dtype=np.int32)
        cnt = np.zeros((G, NCOUNTERS), dtype=np.uint64)
        fS = np.zeros((p, self.nv), dtype=np.uint8)
        ff = np.zeros(p, dtype=np.int32)
        uid = np.zeros(p, dtype=np.uint64)
        hist = np.zeros((p, HMAX), dtype=np.uint64)
        hc = np.zeros(p, dtype=np.int32)
        off = np.zeros((p, self.nv), dtype=np.uint8)
        best = np.zeros(max(self.nv, 1), dtype=np.uint8)
        st = (ctypes.c_void_p * 5)(*[a.ctypes.data for a in (uid, hist, hc, off, best)])
        P = np.ascontiguousarray(params, dtype=np.int64)
        gens = lib().orc_run_state(self.h, _ptr(P), p, G, seed, _ptr(grid), _ptr(filled),
                                   _ptr(bf), _ptr(cnt), _ptr(fS), _ptr(ff), ctypes.byref(st))
        if gens < 0:
            raise ValueError("bad run arguments")
        return dict(grid=grid, filled=int(filled[0]), best_f=bf, counters=cnt, gens=int(gens),
                    final_S=fS, final_f=ff, uid=uid, hist=hist, hcount=hc, offspring=off,
                    best=best[: self.nv])


def distances(A, B) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.uint8)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    D = np.zeros((A.shape[0], B.shape[0]), dtype=np.int32)
    lib().orc_distances(A.shape[1], A.shape[0], _ptr(A), B.shape[0], _ptr(B), _ptr(D))
    return D


def select(nv: int, p: int, spacing: int, seed: int, gen: int, f_all, D_all) -> np.ndarray:
    f_all = np.ascontiguousarray(f_all, dtype=np.int32)
    D_all = np.ascontiguousarray(D_all, dtype=np.int32)
    acc = np.zeros(p, dtype=np.int32)
    lib().orc_select(nv, p, spacing, seed, gen, _ptr(f_all), _ptr(D_all), _ptr(acc))
    return acc


def match(D, uid, hist, hcount, hlen: int = 64, mode: int = M_NEAREST, seed: int = 0,
          gen: int = 0):
    """Returns (partner, dpart, hist', hcount')."""
    p = D.shape[0]
    D = np.ascontiguousarray(D, dtype=np.int32)
    uid = np.ascontiguousarray(uid, dtype=np.uint64)
    hist = np.array(hist, dtype=np.uint64, copy=True).reshape(p, HMAX)
    hcount = np.array(hcount, dtype=np.int32, copy=True)
    partner = np.zeros(p, dtype=np.int32)
    dpart = np.zeros(p, dtype=np.int32)
    lib().orc_match_mode(p, _ptr(D), _ptr(uid), _ptr(hist), _ptr(hcount), hlen, mode, seed, gen,
                         _ptr(partner), _ptr(dpart))
    return partner, dpart, hist, hcount


def aux_threshold(beta_num: int, beta_den: int, D: int, nv: int) -> int:
    return int(lib().orc_aux_threshold(beta_num, beta_den, D, nv))


def aux(seed: int, gen: int, S, partner, dpart, beta_num: int = 20, beta_den: int = 1,
        mode: int = X_AUX):
    S = np.ascontiguousarray(S, dtype=np.uint8)
    p, nv = S.shape
    out = np.zeros_like(S)
    partner = np.ascontiguousarray(partner, dtype=np.int32)
    dpart = np.ascontiguousarray(dpart, dtype=np.int32)
    lib().orc_aux_mode(nv, p, seed, gen, beta_num, beta_den, mode, _ptr(S), _ptr(partner),
                       _ptr(dpart), _ptr(out))
    return out
