"""Independent definitional re-implementations used to pin the oracle.

Pure Python, written straight from the paper's definitions: no conflict
table, no incremental evaluation -- every quantity is recomputed from the
definition each time it is needed.  Slow on purpose; used on tiny inputs.
Shares no code with oracle/ or with the GPU library.
"""

from __future__ import annotations

from fractions import Fraction

M32 = 0xFFFFFFFF


# --- Philox4x32-10 (Salmon et al., SC'11), third independent copy ---------------
def philox4x32_10(ctr, key):
    x = [c & M32 for c in ctr]
    k0, k1 = key[0] & M32, key[1] & M32
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        p0 = 0xD2511F53 * x[0]
        p1 = 0xCD9E8D57 * x[2]
        x = [((p1 >> 32) ^ x[1] ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ x[3] ^ k1) & M32, p0 & M32]
    return x


def fmix32(h):
    h &= M32
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & M32
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & M32
    h ^= h >> 16
    return h


def tie16(wv, wk, v, k):
    """Tie value of move (v, k): top 16 bits of fmix32(wv ^ v) xor fmix32(wk ^ k)."""
    return (fmix32(wv ^ v) ^ fmix32(wk ^ k)) >> 16


def draw(seed, slot, gen, tag, idx):
    return philox4x32_10([0, slot, ((gen << 8) | tag) & M32, idx], [seed & M32, seed >> 32])


# --- Latin square graph (Section 2.1) -------------------------------------------
def reduced_graph(grid):
    """Vertices (row-major empty cells that can take a symbol) and D*(v)."""
    n = len(grid)
    verts, dom, impossible = [], [], 0
    for i in range(n):
        for j in range(n):
            if grid[i][j]:
                continue
            used = {grid[i][t] for t in range(n)} | {grid[t][j] for t in range(n)}
            d = [k for k in range(1, n + 1) if k not in used]
            if d:
                verts.append((i, j))
                dom.append(d)
            else:
                impossible += 1
    return verts, dom, impossible


def adjacent(a, b):
    return a != b and (a[0] == b[0] or a[1] == b[1])


def f_of(S):
    return sum(1 for s in S if s == 0)


def c_of(S, verts):
    """Number of conflicting edges (Eq. 3-4)."""
    c = 0
    for a in range(len(verts)):
        for b in range(a + 1, len(verts)):
            if S[a] and S[a] == S[b] and adjacent(verts[a], verts[b]):
                c += 1
    return c


def conflicting(S, verts, v):
    return S[v] != 0 and any(S[u] == S[v] and adjacent(verts[u], verts[v]) for u in range(len(verts)))


def brute_force_optimum(grid):
    """Maximum number of filled cells over all legal extensions (DFS with a bound)."""
    n = len(grid)
    verts, dom, _ = reduced_graph(grid)
    pre = sum(1 for i in range(n) for j in range(n) if grid[i][j])
    best = [0]
    S = [0] * len(verts)

    def rec(t, filled):
        if filled + (len(verts) - t) <= best[0]:
            return
        if t == len(verts):
            best[0] = max(best[0], filled)
            return
        for k in dom[t]:
            if all(not (S[u] == k and adjacent(verts[u], verts[t])) for u in range(t)):
                S[t] = k
                rec(t + 1, filled + 1)
                S[t] = 0
        rec(t + 1, filled)

    rec(0, 0)
    return pre + best[0]


# --- PLITS re-derived by brute force (Section 3.3, Alg. 3) ------------------------
COUNTERS = ["iters", "moves", "idle", "cands", "elig", "nupd", "snaps", "repairs", "cupd"]


def plits_trace_bruteforce(grid, S_in, seed, slot, gen, depth1, depth2, counters=None):
    """Every iteration's chosen move, re-derived by evaluating F(S') from scratch
    for every neighbour S' of N(S) = N_0(S) u N_c(S).  Returns (rows, S_out).

    counters (a dict, optional) receives the work counts by their definitions:
    iterations with a non-empty neighbourhood, moves, idle iterations, the
    candidate moves examined and eligible vertices per iteration, the
    conflict-table entries a move changes (one per neighbour of the moved
    vertex and coloured end, Section 3.3), the row/column counts it changes
    (two per coloured end), best snapshots and repair uncolourings."""
    verts, dom, _ = reduced_graph(grid)
    n = len(grid)
    nv = len(verts)
    S = list(S_in)
    rows = []
    cnt = {k: 0 for k in COUNTERS}
    for phase, iters in ((1, depth1), (2, depth2)):
        phi = Fraction(1, 2) if phase == 1 else Fraction(nv)
        scale = 2 if phase == 1 else 1  # F is compared as scale * (f + phi c)

        def F(X):
            return int(scale * (f_of(X) + phi * c_of(X, verts)))

        tag = 0x11 if phase == 1 else 0x12
        Fbest = F(S)
        Sbest = list(S)
        tabu = {}
        for it in range(iters):
            elig = [v for v in range(nv) if S[v] == 0 or conflicting(S, verts, v)]
            if not elig:
                break
            cnt["iters"] += 1
            cnt["elig"] += len(elig)
            w = draw(seed, slot, gen, tag, it)
            Fc = F(S)
            best = None
            for v in elig:
                for k in [0] + dom[v]:
                    if k == S[v]:
                        continue
                    cnt["cands"] += 1
                    S2 = list(S)
                    S2[v] = k
                    delta = F(S2) - Fc
                    if not (it >= tabu.get((v, k), 0) or Fc + delta < Fbest):
                        continue
                    key = (delta, tie16(w[1], w[2], v, k), v * (n + 1) + k)
                    if best is None or key < best[0]:
                        best = (key, v, k, delta)
            if best is None:
                rows.append((phase, it, -1, -1, 0, Fc, 1))
                cnt["idle"] += 1
                continue
            _, v, k, delta = best
            old = S[v]
            S[v] = k
            ends = int(old != 0) + int(k != 0)
            cnt["moves"] += 1
            cnt["nupd"] += ends * sum(1 for u in range(nv) if adjacent(verts[u], verts[v]))
            cnt["cupd"] += 2 * ends
            mp = sum(1 for u in range(nv) if S[u] == 0 or conflicting(S, verts, u))
            T = ((w[0] * 10) >> 32) + (6 * mp) // 10
            tabu[(v, old)] = it + 1 + T
            Fn = F(S)
            rows.append((phase, it, v, k, delta, Fn, 0))
            if Fn < Fbest:
                Fbest = Fn
                Sbest = list(S)
                cnt["snaps"] += 1
        S = Sbest
    # final legality guard (Section 3.7): uncolour the most conflicting vertex first
    while True:
        cnts = [sum(1 for u in range(nv) if S[v] and S[u] == S[v] and adjacent(verts[u], verts[v]))
                for v in range(nv)]
        m = max(cnts) if cnts else 0
        if m == 0:
            break
        S[cnts.index(m)] = 0
        cnt["repairs"] += 1
    if counters is not None:
        counters.update(cnt)
    return rows, S


def repair_greedy(S, verts):
    """Section 3.7: uncolour the most conflicting vertex first (lowest id on
    ties) until no conflict is left."""
    S = list(S)
    nv = len(verts)
    while True:
        cnts = [sum(1 for u in range(nv) if S[v] and S[u] == S[v] and adjacent(verts[u], verts[v]))
                for v in range(nv)]
        m = max(cnts) if cnts else 0
        if m == 0:
            return S
        S[cnts.index(m)] = 0


# --- PartialCol re-derived by brute force (Section 3.7) ----------------------------
def partialcol_bruteforce(grid, S_in, seed, slot, gen, depth):
    """Partial-MPMA's search on one offspring: greedy repair, then tabu search
    over legal partial colourings minimising the uncoloured count.  A move
    colours an uncoloured vertex v with k in D*(v) and uncolours v's neighbours
    coloured k, which may not take k back for T = L + 6 f / 10 iterations
    (f after the move) unless that beats the best f.  Every move's value is
    recomputed from scratch.  Returns the best colouring found."""
    verts, dom, _ = reduced_graph(grid)
    n = len(grid)
    nv = len(verts)
    S = repair_greedy(S_in, verts)
    fbest = f_of(S)
    Sbest = list(S)
    tabu = {}
    for it in range(depth):
        U = [v for v in range(nv) if S[v] == 0]
        if not U:
            break
        w = draw(seed, slot, gen, 0x13, it)
        fc = f_of(S)
        best = None
        for v in U:
            for k in dom[v]:
                S2 = list(S)
                S2[v] = k
                for u in range(nv):
                    if S2[u] == k and adjacent(verts[u], verts[v]):
                        S2[u] = 0
                delta = f_of(S2) - fc
                if not (it >= tabu.get((v, k), 0) or fc + delta < fbest):
                    continue
                key = (delta, tie16(w[1], w[2], v, k), v * (n + 1) + k)
                if best is None or key < best[0]:
                    best = (key, v, k, S2)
        if best is None:
            continue
        _, v, k, S2 = best
        gone = [u for u in range(nv) if S[u] == k and adjacent(verts[u], verts[v])]
        S = S2
        assert c_of(S, verts) == 0
        T = ((w[0] * 10) >> 32) + (6 * f_of(S)) // 10
        for u in gone:
            tabu[(u, k)] = it + 1 + T
        if f_of(S) < fbest:
            fbest = f_of(S)
            Sbest = list(S)
    return Sbest


# --- Population update, Alg. 4, transcribed literally ------------------------------
def alg4_literal(f_all, D_all, nv, p, gamma, seed, gen):
    """Alg. 4 with its two fixes: a candidate leaves P^all once examined, and a
    short population is completed with rejected candidates in examination order.
    e(S) = f(S); ties in e are broken by the SELECT draw, then by index."""
    m = 2 * p

    def key(x):
        return (f_all[x], draw(seed, 0, gen, 0x21, x >> 2)[x & 3], x)

    P_all = list(range(m))
    P_next, rejected = [], []
    s_best = min(P_all, key=key)
    P_next.append(s_best)
    P_all.remove(s_best)
    while len(P_next) < p and P_all:
        s_best = min(P_all, key=key)
        dist = min(D_all[s_best][a] for a in P_next)
        if dist > Fraction(nv, gamma):
            P_next.append(s_best)
        else:
            rejected.append(s_best)
        P_all.remove(s_best)
    for x in rejected:
        if len(P_next) >= p:
            break
        P_next.append(x)
    return P_next


# --- Initial population (Section 3.2, reading A), from its definition --------------
def init_literal(grid, seed, slot):
    """Randomised greedy legal colouring: vertices in the order of their
    INIT_ORDER draws (ties by id), each takes the colour of D*(v) unused by its
    already coloured neighbours drawn by INIT_PICK, or stays uncoloured."""
    verts, dom, _ = reduced_graph(grid)
    nv = len(verts)
    order = sorted(range(nv), key=lambda v: (draw(seed, slot, 0, 0x01, v >> 2)[v & 3], v))
    S = [0] * nv
    for t, v in enumerate(order):
        legal = [k for k in dom[v]
                 if not any(S[u] == k and adjacent(verts[u], verts[v]) for u in range(nv))]
        if legal:
            S[v] = legal[(draw(seed, slot, 0, 0x02, t)[0] * len(legal)) >> 32]
    return S


def aux_threshold_exact(beta_num, beta_den, D, nv):
    """Eq. 9 scaled to a 32-bit draw: floor(p_ij 2^32) with p_ij = 1 - |V| / (beta D),
    beta = beta_num / beta_den; 0 when p_ij <= 0 (reading R).  Exact rationals."""
    if D == 0:
        return 0
    pij = 1 - Fraction(nv * beta_den, beta_num * D)
    if pij <= 0:
        return 0
    return (pij.numerator << 32) // pij.denominator


# --- The memetic algorithm, Alg. 2, transcribed literally --------------------------
def mpma_literal(grid, p, G, seed, depth1, depth2, hist_len=64, beta=(20, 1), gamma=10):
    """Alg. 2 step by step on lists.  P_1 = randomised greedy colourings; in
    generation 1 the offspring are P_1 itself.  Each generation: PLITS on every
    offspring (slot i, generation g), best-solution saving (lowest slot among
    equal f, strict improvement), distances over P_t then P', Alg. 4, uids
    (initial individuals: their slot; offspring of generation g: g << 32 | slot;
    survivors keep theirs), nearest-neighbour matching that skips the uids of
    recent partners (history of the last hist_len partners, oldest dropped
    first, carried by the individual; offspring start with an empty one; the
    filter is dropped when it excludes everyone) and the AUX crossover.
    Returns the final population with f, uids, histories (oldest first), the
    offspring waiting for the next search, S* and the best f per generation."""
    import numpy as np

    verts, dom, _ = reduced_graph(grid)
    nv = len(verts)
    P = [init_literal(grid, seed, i) for i in range(p)]
    f = [f_of(S) for S in P]
    uid = list(range(p))
    hist = [[] for _ in range(p)]
    O = [list(S) for S in P]
    star, fstar, best_f = None, None, []
    for g in range(1, G + 1):
        Pp = [plits_trace_bruteforce(grid, O[i], seed, i, g, depth1, depth2)[1] for i in range(p)]
        fp = [f_of(S) for S in Pp]
        b = min(range(p), key=lambda i: (fp[i], i))
        if fstar is None or fp[b] < fstar:
            fstar, star = fp[b], list(Pp[b])
        best_f.append(fstar)
        A = P + Pp
        fa = f + fp
        D = [[sum(1 for v in range(nv) if A[x][v] != A[y][v]) for y in range(2 * p)]
             for x in range(2 * p)]
        acc = alg4_literal(fa, D, nv, p, gamma, seed, g)
        uid_all = uid + [(g << 32) | i for i in range(p)]
        hist_all = hist + [[] for _ in range(p)]
        P = [list(A[x]) for x in acc]
        f = [fa[x] for x in acc]
        uid = [uid_all[x] for x in acc]
        hist = [list(hist_all[x]) for x in acc]
        Dn = np.array([[D[acc[i]][acc[j]] for j in range(p)] for i in range(p)])
        partner = []
        for i in range(p):
            allowed = np.array([j != i and uid[j] not in hist[i] for j in range(p)])
            if not allowed.any():
                allowed = np.array([j != i for j in range(p)])
            j = int(np.argmin(np.where(allowed, Dn[i], np.iinfo(np.int64).max)))
            partner.append(j)
            if hist_len > 0:
                hist[i].append(uid[j])
                if len(hist[i]) > hist_len:
                    hist[i].pop(0)
        O = []
        for i, j in enumerate(partner):
            thr = aux_threshold_exact(beta[0], beta[1], int(Dn[i][j]), nv)
            O.append([P[i][v] if draw(seed, i, g, 0x31, v >> 2)[v & 3] < thr else P[j][v]
                      for v in range(nv)])
    return dict(P=P, f=f, uid=uid, hist=hist, O=O, star=star, best_f=best_f)
