"""Pins of the oracle's whole-run bookkeeping (Alg. 2), of its work counters
and of the AUX threshold (Eq. 9).

The whole run is compared with a literal Python transcription of Alg. 2
(tests/refdefs.py) that builds every step from its definition: the
brute-force tabu search, Alg. 4 as printed (with the termination fix),
numpy masked-argmin matching with partner histories as lists, and the
crossover with an exact rational threshold.  Planted slips in a copy of the
oracle's run loop must make the comparison fail.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2103_10453_amd import instances as gen
from tests import refdefs as R

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "mpma_oracle.c")

# (n, prefill, grid seed, population, generations, depth1, depth2, history length)
RUN_CASES = [
    (4, 0.3, 12, 4, 4, 10, 6, 64),   # p = 4: histories exclude everyone -> fallback
    (5, 0.4, 0, 6, 3, 12, 6, 64),
    (5, 0.3, 7, 8, 3, 10, 6, 2),     # history of 2: FIFO eviction
    (4, 0.4, 65, 5, 3, 14, 6, 1),
]


def _hist_list(hist_row, hcount, hlen):
    """Partner uids of one individual, oldest first, from the oracle's ring."""
    if hlen == 0:
        return []
    if hcount <= hlen:
        return [int(x) for x in hist_row[:hcount]]
    pos = hcount % hlen
    return [int(x) for x in list(hist_row[pos:hlen]) + list(hist_row[:pos])]


def _params(oracle_mod, I, d1, d2, hlen):
    P = I.params()
    P[oracle_mod.P_DEPTH1], P[oracle_mod.P_DEPTH2] = d1, d2
    P[oracle_mod.P_HIST] = hlen
    return P


def _compare(st, ref, nv, hlen):
    """Mismatching parts of an oracle run state against the transcription."""
    bad = []
    if [list(map(int, r)) for r in st["final_S"]] != ref["P"]:
        bad.append("population")
    if list(map(int, st["final_f"])) != ref["f"]:
        bad.append("f")
    if list(map(int, st["uid"])) != ref["uid"]:
        bad.append("uid")
    hists = [_hist_list(st["hist"][i], int(st["hcount"][i]), hlen) for i in range(len(ref["P"]))]
    if hists != ref["hist"]:
        bad.append("history")
    if [list(map(int, r)) for r in st["offspring"]] != ref["O"]:
        bad.append("offspring")
    if list(map(int, st["best"][:nv])) != ref["star"]:
        bad.append("best")
    if list(map(int, st["best_f"])) != ref["best_f"]:
        bad.append("best_f")
    return bad


@pytest.fixture(scope="module")
def literal_runs():
    out = {}
    for case in RUN_CASES:
        n, r, gs, p, G, d1, d2, hlen = case
        g = gen.random_greedy(n, r, gs)
        seed = (1 << 35) + 1000 * gs + p
        out[case] = (g, seed, R.mpma_literal(g.tolist(), p, G, seed, d1, d2, hist_len=hlen))
    return out


@pytest.mark.parametrize("case", RUN_CASES)
def test_run_equals_literal_alg2(oracle_mod, literal_runs, case):
    """Alg. 2 (Section 3.1): population, f, uids, partner histories, the
    offspring of the next generation, S* and the best f of every generation
    equal the literal transcription after G generations."""
    n, r, gs, p, G, d1, d2, hlen = case
    g, seed, ref = literal_runs[case]
    I = oracle_mod.Instance(g)
    st = I.run_state(_params(oracle_mod, I, d1, d2, hlen), p, G, seed)
    assert st["gens"] == G
    assert _compare(st, ref, I.nv, hlen) == []


def test_run_cases_exercise_the_bookkeeping(literal_runs):
    """The cases contain survivors of P_t next to new offspring, histories
    that exclude every other individual, and full FIFOs that drop partners."""
    survivors = fallback = evicted = 0
    for case, (g, seed, ref) in literal_runs.items():
        p, G, hlen = case[3], case[4], case[7]
        survivors += sum(1 for u in ref["uid"] if (u >> 32) < G)
        fallback += sum(1 for i in range(p) if len(set(ref["hist"][i])) >= p - 1)
        evicted += sum(1 for h in ref["hist"] if hlen and len(h) == hlen)
    assert survivors > 0 and fallback > 0 and evicted > 0


# Slips in the run loop of Alg. 2 that the outcome tests (planted grids
# complete, tiny grids reach their optimum, determinism) do not see.
MUTATIONS = {
    "survivors drop their history": ("hcn[r] = hc[x];", "hcn[r] = 0;"),
    "offspring uids by rank": ("uidn[r] = uid[x];",
                               "uidn[r] = (x >= p) ? (((uint64_t)g << 32) | (uint32_t)r) : uid[x];"),
    "history row of the wrong individual": (
        "memcpy(histn + (size_t)r * ORC_HMAX, hist + (size_t)x * ORC_HMAX,",
        "memcpy(histn + (size_t)r * ORC_HMAX, hist + (size_t)r * ORC_HMAX,"),
    "distance columns not re-indexed": ("Dn[(size_t)i * p + j] = Dall[(size_t)acc[i] * m + acc[j]];",
                                        "Dn[(size_t)i * p + j] = Dall[(size_t)acc[i] * m + j];"),
    "first offspring not the initial population": (
        "memcpy(Soff, Sall, (size_t)p * snv);", "memset(Soff, 0, (size_t)p * snv);"),
    "best saving keeps the last of equal f": ("if (fall[p + i] < fall[p + b]) b = i;",
                                              "if (fall[p + i] <= fall[p + b]) b = i;"),
    "offspring uids not reset": ("uid[p + i] = ((uint64_t)g << 32) | (uint32_t)i;",
                                 "uid[p + i] = (uint64_t)i;"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, f"mutation site not found: {name}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    hdr = os.path.join(os.path.dirname(ORACLE_SRC), "mpma_oracle.h")
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-I", os.path.dirname(hdr), "-o", str(so), str(path)])
    return ctypes.CDLL(str(so))


def _mutant_state(L, oracle_mod, g, P, p, G, seed):
    V = ctypes.c_void_p
    L.orc_create.restype = V
    L.orc_create.argtypes = [ctypes.c_int32, V, V]
    L.orc_info.argtypes = [V, V]
    L.orc_run_state.restype = ctypes.c_int32
    L.orc_run_state.argtypes = [V, V, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64] + [V] * 7
    L.orc_destroy.argtypes = [V]
    g = np.ascontiguousarray(g, dtype=np.int8)
    status = np.zeros(1, dtype=np.int32)
    h = L.orc_create(g.shape[0], g.ctypes.data, status.ctypes.data)
    info = np.zeros(4, dtype=np.int32)
    L.orc_info(h, info.ctypes.data)
    nv = int(info[0])
    n = g.shape[0]
    arrs = dict(grid=np.zeros((n, n), np.int8), filled=np.zeros(1, np.int32),
                best_f=np.zeros(G, np.int32), counters=np.zeros((G, oracle_mod.NCOUNTERS), np.uint64),
                final_S=np.zeros((p, nv), np.uint8), final_f=np.zeros(p, np.int32),
                uid=np.zeros(p, np.uint64), hist=np.zeros((p, oracle_mod.HMAX), np.uint64),
                hcount=np.zeros(p, np.int32), offspring=np.zeros((p, nv), np.uint8),
                best=np.zeros(max(nv, 1), np.uint8))
    st = (ctypes.c_void_p * 5)(*[arrs[k].ctypes.data for k in ("uid", "hist", "hcount",
                                                                 "offspring", "best")])
    P = np.ascontiguousarray(P, dtype=np.int64)
    L.orc_run_state(h, P.ctypes.data, p, G, seed, *[arrs[k].ctypes.data for k in
                    ("grid", "filled", "best_f", "counters", "final_S", "final_f")],
                    ctypes.byref(st))
    L.orc_destroy(h)
    return arrs, nv


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_bookkeeping_slips_are_caught(oracle_mod, literal_runs, tmp_path, name):
    """Each slip, planted in a copy of the oracle, makes at least one whole
    run differ from the literal transcription of Alg. 2."""
    old, new = MUTATIONS[name]
    L = _build_mutant(tmp_path, name, old, new)
    caught = False
    for case, (g, seed, ref) in literal_runs.items():
        n, r, gs, p, G, d1, d2, hlen = case
        P = oracle_mod.default_params(0, n)
        P[oracle_mod.P_DEPTH1], P[oracle_mod.P_DEPTH2] = d1, d2
        P[oracle_mod.P_HIST] = hlen
        st, nv = _mutant_state(L, oracle_mod, g, P, p, G, seed)
        if _compare(st, ref, nv, hlen):
            caught = True
            break
    assert caught, f"planted slip not detected: {name}"


# --- work counters --------------------------------------------------------------------
CNT_CASES = [(4, 0.3, 12), (5, 0.4, 0), (5, 0.6, 1), (5, 0.4, 303), (4, 0.5, 302)]


@pytest.mark.parametrize("n,r,gseed", CNT_CASES)
def test_counters_equal_their_definitions(oracle_mod, n, r, gseed):
    """Every counter of one search equals its definition counted on the
    brute-force move trace: iterations, moves, idle iterations, candidates
    examined, eligible vertices, conflict-table entries updated (Section 3.3:
    the neighbours of the moved vertex, once per coloured end), row/column
    counts updated, snapshots and repair uncolourings."""
    g = gen.random_greedy(n, r, gseed)
    I = oracle_mod.Instance(g)
    rng = np.random.default_rng(gseed)
    _, dom, _ = R.reduced_graph(g.tolist())
    S0 = np.array([rng.choice([0] + d) for d in dom], dtype=np.uint8)
    P = I.params(depth=60 + 2 * I.nv)
    seed64 = (1 << 33) + 17 * gseed
    _, _, cnt = I.plits(P, seed64, 3, [5], S0)
    ref = {}
    R.plits_trace_bruteforce(g.tolist(), list(S0), seed64, 5, 3, int(P[0]), int(P[1]),
                             counters=ref)
    assert dict(zip(oracle_mod.COUNTER_NAMES, map(int, cnt[0]))) == ref
    assert ref["nupd"] > ref["cupd"] > 0


def test_partialcol_neighbour_updates(oracle_mod):
    """PartialCol (Section 3.7): a move changes conf[u][k] of every neighbour u
    of the coloured vertex and of every neighbour of each vertex it uncolours;
    summed over the search this is at least the row/column count changes and
    at most deg_max times them."""
    g = gen.random_greedy(12, 0.6, 2)
    I = oracle_mod.Instance(g)
    verts, dom, _ = R.reduced_graph(g.tolist())
    deg = [sum(1 for u in verts if R.adjacent(u, v)) for v in verts]
    S, _ = I.init(3, 4)
    P = I.params(depth=600, variant=oracle_mod.V_PARTIAL)
    _, _, cnt = I.plits(P, 3, 1, list(range(4)), S)
    c = dict(zip(oracle_mod.COUNTER_NAMES, cnt.sum(0)))
    assert c["moves"] > 0
    assert c["cupd"] >= 2 * c["moves"]
    assert c["cupd"] // 2 * min(deg) <= c["nupd"] <= c["cupd"] // 2 * max(deg)


# --- AUX threshold (Eq. 9) ------------------------------------------------------------
@pytest.mark.parametrize("bn,bd,D,nv", [
    (20, 1, 700, 3430), (20, 1, 100, 1250), (20, 1, 62, 1250), (20, 1, 63, 1250),
    (1000000, 666667, 3400, 3430), (1000000, 1, 16129, 16129), (999999, 7, 4000, 4900),
    (3, 2, 5, 7), (20, 1, 0, 60)])
def test_aux_threshold_is_exact(oracle_mod, bn, bd, D, nv):
    """floor(p_ij 2^32) with p_ij = 1 - |V| / (beta D) (Eq. 9), 0 when p_ij <= 0,
    as an exact rational -- also where (beta_num D - beta_den |V|) 2^32
    exceeds 64 bits (large beta terms at n >= 70)."""
    assert oracle_mod.aux_threshold(bn, bd, D, nv) == R.aux_threshold_exact(bn, bd, D, nv)


def test_aux_children_follow_the_exact_threshold(oracle_mod):
    """With a large beta (1000000/666667) at n = 70 sizes the child takes the
    first parent's colour exactly where the XOVER draw is below the exact
    threshold."""
    nv, p, seed, gen_ = 3430, 3, 77, 4
    S = np.zeros((p, nv), dtype=np.uint8)
    S[1] = 1
    S[2] = 2
    partner = np.array([1, 2, 0], dtype=np.int32)
    dpart = np.array([3400, 1200, 3430], dtype=np.int32)
    out = oracle_mod.aux(seed, gen_, S, partner, dpart, beta_num=1000000, beta_den=666667)
    for i in range(p):
        thr = R.aux_threshold_exact(1000000, 666667, int(dpart[i]), nv)
        for v in range(0, nv, 97):
            w = R.draw(seed, i, gen_, 0x31, v >> 2)[v & 3]
            assert out[i, v] == (S[i, v] if w < thr else S[partner[i], v])
