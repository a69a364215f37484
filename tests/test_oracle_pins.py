"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  A mistake anywhere in the oracle (a
dropped term, a wrong sign, a swapped index, a wrong tie-break or tenure)
breaks at least one of them.
"""

import os

import numpy as np
import pytest

from paper_2103_10453_amd import instances as gen
from tests import refdefs as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --- randomness --------------------------------------------------------------------
def test_philox_known_answers(oracle_mod):
    """Philox4x32-10 against the published known-answer vectors (Salmon et al.)."""
    for row in _read_golden("philox4x32_10_kat.txt"):
        vals = [int(x, 16) for x in row]
        ctr, key, want = vals[:4], vals[4:6], vals[6:10]
        assert list(oracle_mod.philox(ctr, key)) == want
        assert R.philox4x32_10(ctr, key) == want


def test_fmix32_published_values_and_bijection(oracle_mod):
    """fmix32 = MurmurHash3 finaliser: published empty-input hashes, and exact
    inversion with the modular inverses of its multipliers (a bijection, so the
    tie keys of distinct candidates never collide)."""
    for seed_hex, want_hex in _read_golden("murmur3_fmix32.txt"):
        assert oracle_mod.fmix32(int(seed_hex, 16)) == int(want_hex, 16)
    inv1 = pow(0x85EBCA6B, -1, 1 << 32)
    inv2 = pow(0xC2B2AE35, -1, 1 << 32)

    def unshift(h, s):
        x = h
        for _ in range(32 // s + 1):
            x = h ^ (x >> s)
        return x & 0xFFFFFFFF

    rng = np.random.default_rng(1)
    for x in list(rng.integers(0, 1 << 32, size=2000, dtype=np.uint64)) + [0, 1, 0xFFFFFFFF]:
        x = int(x)
        h = oracle_mod.fmix32(x)
        y = unshift(h, 16)
        y = (y * inv2) & 0xFFFFFFFF
        y = unshift(y, 13)
        y = (y * inv1) & 0xFFFFFFFF
        y = unshift(y, 16)
        assert y == x


def test_tie_values_are_fair(oracle_mod):
    """Best-move ties (Section 3.3, a best move is taken; ties at random): the
    tie value of a move is 16 bits; over random tie words every one of
    three tied moves comes first about a third of the time, whether they
    are colours of one vertex, one colour on three vertices, or mixed, and
    two moves share a value only rarely (then the smaller move id wins)."""
    rng = np.random.default_rng(5)
    words = [(int(a), int(b)) for a, b in rng.integers(0, 1 << 32, size=(6000, 2), dtype=np.uint64)]
    for wv, wk in words[:50]:
        for v, k in ((0, 0), (1249, 50), (16128, 127)):
            assert 0 <= oracle_mod.tie16(wv, wk, v, k) < 1 << 16
    for moves in (((7, 1), (7, 2), (7, 3)),          # colours of one vertex
                  ((3, 5), (4, 5), (900, 5)),        # one colour, three vertices
                  ((3, 5), (3, 6), (4, 5))):         # mixed
        wins = [0, 0, 0]
        for wv, wk in words:
            t = [oracle_mod.tie16(wv, wk, v, k) for v, k in moves]
            wins[int(np.argmin(t))] += 1
        assert all(abs(x / len(words) - 1 / 3) < 0.03 for x in wins), (moves, wins)
    eq = sum(oracle_mod.tie16(wv, wk, 3, 5) == oracle_mod.tie16(wv, wk, 3, 6) for wv, wk in words)
    assert eq <= 3


def test_philox_uniformity_chi2(oracle_mod):
    """Sanity: the top 4 bits of 16384 draws are close to uniform (chi^2, 15 dof)."""
    counts = np.zeros(16)
    for i in range(4096):
        for w in oracle_mod.philox([0, i, 0x111, 7], [12345, 678]):
            counts[int(w) >> 28] += 1
    exp = counts.sum() / 16
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 45  # p ~ 1e-4 for 15 dof


# --- instance and preprocessing (Alg. 1, Section 2.2) ---------------------------------
def test_worked_example_n3(oracle_mod):
    rows = {r[0]: r[1:] for r in _read_golden("plse_n3_example.txt") if r[0] != "grid"}
    grid = np.array([[int(x) for x in r[1:]] for r in _read_golden("plse_n3_example.txt")
                     if r[0] == "grid"], dtype=np.int8)
    I = oracle_mod.Instance(grid)
    assert I.l == int(rows["l"][0])
    assert I.ub == int(rows["ub"][0])
    assert R.brute_force_optimum(grid.tolist()) == int(rows["optimum"][0])
    vr, vc, off, dom = I.tables()
    cells = [int(a) * 3 + int(b) for a, b in zip(vr, vc)]
    assert int(rows["impossible_cell"][0]) not in cells and grid.flat[6] == 0
    v6 = cells.index(5)
    assert list(dom[off[v6]:off[v6 + 1]]) == [int(rows["domain_of_cell_5"][0])]
    # any relabelling of symbols, rows or columns gives the same l and UB
    perm = np.array([0, 3, 1, 2], dtype=np.int8)
    I2 = oracle_mod.Instance(perm[grid][::-1, :].T.copy())
    assert (I2.l, I2.ub) == (I.l, I.ub)


@pytest.mark.parametrize("n,r,seed", [(5, 0.3, 1), (7, 0.5, 2), (10, 0.4, 3), (50, 0.5, 1000)])
def test_planted_has_no_impossible_cells(oracle_mod, n, r, seed):
    g = gen.planted(n, r, seed)
    assert gen.is_partial_latin(g)
    I = oracle_mod.Instance(g)
    assert I.l == 0 and I.ub == n * n
    assert I.nv == int(round((1 - r) * n * n))


@pytest.mark.parametrize("seed", range(12))
def test_domains_and_bound_by_definition(oracle_mod, seed):
    """D*(v), l and UB against the definitions; the brute-force optimum never
    exceeds UB (n^2 - l, or n^2 - 2 when l = 1)."""
    n = 3 + seed % 3
    g = gen.random_greedy(n, 0.45 + 0.05 * (seed % 4), 77 + seed)
    I = oracle_mod.Instance(g)
    verts, dom, imp = R.reduced_graph(g.tolist())
    vr, vc, off, d = I.tables()
    assert list(zip(vr, vc)) == verts
    assert [list(d[off[v]:off[v + 1]]) for v in range(I.nv)] == dom
    assert I.l == imp
    assert I.ub == (n * n - 2 if imp == 1 else n * n - imp)
    assert R.brute_force_optimum(g.tolist()) <= I.ub


def test_invalid_grids_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.Instance(np.array([[1, 1], [0, 0]], dtype=np.int8))
    with pytest.raises(ValueError):
        oracle_mod.Instance(np.array([[1, 0], [1, 0]], dtype=np.int8))
    with pytest.raises(ValueError):
        oracle_mod.Instance(np.array([[3, 0], [0, 0]], dtype=np.int8))


# --- initialisation ---------------------------------------------------------------------
@pytest.mark.parametrize("n,r,planted", [(10, 0.4, True), (12, 0.6, False), (20, 0.3, False)])
def test_init_legal_and_maximal(oracle_mod, n, r, planted):
    g = gen.planted(n, r, 5) if planted else gen.random_greedy(n, r, 5)
    I = oracle_mod.Instance(g)
    verts, dom, _ = R.reduced_graph(g.tolist())
    S, f = I.init(99, 16)
    for i in range(16):
        s = list(S[i])
        assert R.c_of(s, verts) == 0
        assert f[i] == R.f_of(s)
        for v in range(I.nv):
            assert s[v] == 0 or s[v] in dom[v]
            if s[v] == 0:  # maximal: no colour of D*(v) is free
                for k in dom[v]:
                    assert any(s[u] == k and R.adjacent(verts[u], verts[v]) for u in range(I.nv))
    # different slots draw different orders
    assert len({bytes(S[i]) for i in range(16)}) > 1


def test_init_draws_are_uniform_on_a_symmetric_grid(oracle_mod):
    """On the empty grid every cell and symbol are interchangeable, so a random
    greedy colouring with a uniform pick among the legal colours gives every
    symbol probability 1/n at every cell (chi^2 over 3000 colourings)."""
    n = 5
    I = oracle_mod.Instance(np.zeros((n, n), dtype=np.int8))
    S, f = I.init(2024, 3000)
    counts = np.stack([(S == k).sum(0) for k in range(1, n + 1)])  # n x cells
    assert counts.sum() == (S > 0).sum()
    exp = counts.sum(0, keepdims=True) / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    dof = (n - 1) * n * n
    assert chi2 < dof + 6 * np.sqrt(2 * dof)
    # the first vertex coloured is never blocked: every cell is coloured in some slot
    assert np.all((S > 0).any(0))


# --- PLITS --------------------------------------------------------------------------------
# Tiny grids (gseed of gen.random_greedy) that cannot be completed, so the search
# runs its full depth through both phases with uphill moves, tabu-blocked and
# aspirated moves and idle iterations; plus completable ones that end early.
TRACE_CASES = [(4, 0.3, 12), (4, 0.3, 65), (4, 0.4, 10), (4, 0.4, 65), (5, 0.4, 0),
               (5, 0.5, 2), (5, 0.6, 1), (5, 0.6, 0), (5, 0.4, 303), (4, 0.5, 302)]


@pytest.mark.parametrize("n,r,gseed", TRACE_CASES)
def test_plits_moves_match_bruteforce(oracle_mod, n, r, gseed):
    """Every move the oracle takes equals the best admissible one-move found by
    evaluating F(S') from scratch over N(S) (Eq. 6, 7; Alg. 3; tenure and
    aspiration of Section 3.3), including idle iterations and the final repair."""
    g = gen.random_greedy(n, r, gseed)
    I = oracle_mod.Instance(g)
    rng = np.random.default_rng(gseed)
    verts, dom, _ = R.reduced_graph(g.tolist())
    # an arbitrary (conflicting, partial) start so that both neighbourhoods occur
    S0 = np.array([rng.choice([0] + d) for d in dom], dtype=np.uint8)
    P = I.params(depth=60 + 2 * I.nv)
    seed64 = (1 << 33) + 17 * gseed
    rows = I.plits_trace(P, seed64, 3, 5, S0)
    ref_rows, ref_S = R.plits_trace_bruteforce(g.tolist(), list(S0), seed64, 5, 3,
                                               int(P[0]), int(P[1]))
    assert [tuple(int(x) for x in row) for row in rows] == [tuple(x) for x in ref_rows]
    S_out, f_out, _ = I.plits(P, seed64, 3, [5], S0)
    assert list(S_out[0]) == ref_S
    assert R.c_of(list(S_out[0]), verts) == 0


def test_trace_cases_exercise_the_rules(oracle_mod):
    """The hard trace cases do contain idle iterations, uphill moves and phase 2."""
    idle = uphill = phase2 = 0
    for n, r, gseed in TRACE_CASES[:8]:
        g = gen.random_greedy(n, r, gseed)
        I = oracle_mod.Instance(g)
        rng = np.random.default_rng(gseed)
        _, dom, _ = R.reduced_graph(g.tolist())
        S0 = np.array([rng.choice([0] + d) for d in dom], dtype=np.uint8)
        rows = I.plits_trace(I.params(depth=60 + 2 * I.nv), (1 << 33) + 17 * gseed, 3, 5, S0)
        idle += rows[:, 6].sum()
        uphill += (rows[:, 4] > 0).sum()
        phase2 += (rows[:, 0] == 2).sum()
    assert idle > 20 and uphill > 50 and phase2 > 100


@pytest.mark.parametrize("n,r,planted,seed", [(10, 0.4, True, 1), (12, 0.6, False, 2),
                                              (15, 0.5, False, 3), (20, 0.7, False, 4)])
def test_plits_incremental_state_equals_recomputation(oracle_mod, n, r, planted, seed):
    """Paranoid mode recomputes conf, f, c from scratch after every move and
    aborts on any difference; outputs are legal and f is the uncoloured count."""
    g = gen.planted(n, r, seed) if planted else gen.random_greedy(n, r, seed)
    I = oracle_mod.Instance(g)
    verts, _, _ = R.reduced_graph(g.tolist())
    P = I.params(depth=10 * n * n, paranoid=True)
    S, _ = I.init(11, 6)
    S_out, f, cnt = I.plits(P, 11, 1, list(range(6)), S)
    for i in range(6):
        assert R.c_of(list(S_out[i]), verts) == 0
        assert f[i] == R.f_of(list(S_out[i]))
    names = oracle_mod.COUNTER_NAMES
    c = dict(zip(names, cnt.sum(0)))
    assert c["moves"] + c["idle"] == c["iters"]
    assert c["cands"] >= c["iters"] and c["elig"] >= c["iters"]


@pytest.mark.parametrize("n,r,gseed", TRACE_CASES)
def test_partialcol_matches_bruteforce(oracle_mod, n, r, gseed):
    """Partial-MPMA (Section 3.7): repair, then PartialCol; the oracle's result
    equals the brute-force re-derivation that recomputes every move's value
    from the definition."""
    g = gen.random_greedy(n, r, gseed)
    I = oracle_mod.Instance(g)
    rng = np.random.default_rng(gseed)
    verts, dom, _ = R.reduced_graph(g.tolist())
    S0 = np.array([rng.choice([0] + d) for d in dom], dtype=np.uint8)
    depth = 40 + 3 * I.nv
    P = I.params(depth=depth, variant=oracle_mod.V_PARTIAL)
    seed64 = (1 << 34) + 31 * gseed
    S_out, f_out, cnt = I.plits(P, seed64, 2, [3], S0)
    ref = R.partialcol_bruteforce(g.tolist(), list(S0), seed64, 3, 2, depth)
    assert list(S_out[0]) == ref
    assert f_out[0] == R.f_of(ref) and R.c_of(ref, verts) == 0
    assert int(cnt[0, 7]) == R.f_of(R.repair_greedy(list(S0), verts)) - R.f_of(list(S0))


@pytest.mark.parametrize("n,r,seed", [(12, 0.6, 2), (20, 0.7, 4), (15, 0.8, 5)])
def test_partialcol_incremental_state_and_progress(oracle_mod, n, r, seed):
    """Paranoid recomputation after every PartialCol move; outputs legal and
    never worse than the repaired offspring."""
    g = gen.random_greedy(n, r, seed)
    I = oracle_mod.Instance(g)
    verts, dom, _ = R.reduced_graph(g.tolist())
    rng = np.random.default_rng(seed)
    S0 = np.array([[rng.choice([0] + d) for d in dom] for _ in range(4)], dtype=np.uint8)
    P = I.params(depth=10 * n * n, paranoid=True, variant=oracle_mod.V_PARTIAL)
    S_out, f, cnt = I.plits(P, 13, 1, list(range(4)), S0)
    for i in range(4):
        assert R.c_of(list(S_out[i]), verts) == 0
        assert f[i] == R.f_of(list(S_out[i]))
        assert f[i] <= R.f_of(R.repair_greedy(list(S0[i]), verts))


def test_plits_improves_or_keeps_start(oracle_mod):
    """Phase 2 starts from phase 1's best, and a legal start is never made worse:
    with phi = |V| a legal S with f uncoloured has F = f, and F* only decreases."""
    g = gen.random_greedy(20, 0.5, 9)
    I = oracle_mod.Instance(g)
    S, f0 = I.init(5, 8)
    S_out, f1, _ = I.plits(I.params(depth=4000), 5, 1, list(range(8)), S)
    assert np.all(f1 <= f0)


# --- distances, selection, matching, crossover ------------------------------------------
def test_distances_definition(oracle_mod):
    rng = np.random.default_rng(3)
    A = rng.integers(0, 6, size=(9, 37), dtype=np.uint8)
    B = rng.integers(0, 6, size=(7, 37), dtype=np.uint8)
    D = oracle_mod.distances(A, B)
    np.testing.assert_array_equal(D, (A[:, None, :] != B[None, :, :]).sum(-1))


@pytest.mark.parametrize("p,nv,seed", [(4, 20, 1), (16, 30, 2), (32, 50, 3), (64, 40, 4),
                                       (128, 100, 5)])
def test_select_is_algorithm4(oracle_mod, p, nv, seed):
    rng = np.random.default_rng(seed)
    m = 2 * p
    # few distinct f values (many ties) and some close pairs
    X = rng.integers(0, 3, size=(m, nv), dtype=np.uint8)
    for t in range(m // 3):
        a, b = rng.integers(0, m, size=2)
        X[b] = X[a]
        X[b, rng.integers(0, nv, size=rng.integers(0, nv // 8 + 1))] = 2
    D = oracle_mod.distances(X, X)
    f = rng.integers(0, 3, size=m).astype(np.int32)
    acc = oracle_mod.select(nv, p, 10, 1234 + seed, 7, f, D)
    want = R.alg4_literal(f.tolist(), D.tolist(), nv, p, 10, 1234 + seed, 7)
    assert list(acc) == want
    assert len(set(acc.tolist())) == p
    # spacing holds among the members admitted by the scan
    scan = []
    for x in acc:
        if all(10 * D[x, a] > nv for a in scan):
            scan.append(x)
        else:
            break


@pytest.mark.parametrize("seed", range(4))
def test_match_is_masked_argmin(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    p = 24
    D = rng.integers(0, 12, size=(p, p)).astype(np.int32)
    D = np.minimum(D, D.T)
    uid = rng.permutation(1000)[:p].astype(np.uint64)
    hist = np.zeros((p, 64), dtype=np.uint64)
    hc = np.zeros(p, dtype=np.int32)
    for i in range(p):
        k = int(rng.integers(0, p + 2))
        ex = rng.choice(uid, size=min(k, p), replace=False)
        hist[i, :len(ex)] = ex
        hc[i] = len(ex)
    partner, dpart, hist2, hc2 = oracle_mod.match(D, uid, hist, hc)
    for i in range(p):
        mask = np.isin(uid, hist[i, :hc[i]])
        mask[i] = True
        if mask.all():
            mask = np.zeros(p, dtype=bool)
            mask[i] = True
        Dm = np.where(mask, np.iinfo(np.int32).max, D[i])
        assert partner[i] == int(np.argmin(Dm))
        assert dpart[i] == D[i, partner[i]]
        assert hist2[i, hc[i] % 64] == uid[partner[i]] and hc2[i] == hc[i] + 1


def test_match_history_fifo(oracle_mod):
    """After 64 crossovers the oldest partner is forgotten first."""
    p = 70
    D = np.abs(np.arange(p)[:, None] - np.arange(p)[None, :]).astype(np.int32)
    uid = np.arange(p, dtype=np.uint64) + 500
    hist = np.zeros((p, 64), dtype=np.uint64)
    hc = np.zeros(p, dtype=np.int32)
    seen = []
    for t in range(p + 3):
        partner, _, hist, hc = oracle_mod.match(D, uid, hist, hc)
        seen.append(int(partner[0]))
    # slot 0 walks outwards through 1..65; storing 65 evicts the oldest entry (1),
    # which is then the nearest allowed partner again, and so on
    assert seen[:65] == list(range(1, 66))
    assert seen[65:69] == [1, 2, 3, 4]


def test_aux_expected_distances(oracle_mod):
    """Section 3.5.2: E[D(S_i, S_o)] = |V|/beta and E[D(S_j, S_o)] = D_ij - |V|/beta."""
    rng = np.random.default_rng(0)
    nv, beta = 400, 20
    K = 600
    S = rng.integers(1, 9, size=(2 * K, nv), dtype=np.uint8)
    Dij = 150
    for i in range(K):  # partner of child i is row K+i, differing on exactly Dij vertices
        S[K + i] = S[i]
        idx = rng.choice(nv, size=Dij, replace=False)
        S[K + i, idx] = (S[i, idx] % 8) + 1
    partner = np.concatenate([np.arange(K, 2 * K), np.arange(K)]).astype(np.int32)
    dpart = np.full(2 * K, Dij, dtype=np.int32)
    child = oracle_mod.aux(42, 3, S, partner, dpart, beta, 1)[:K]
    assert np.all((child == S[:K]) | (child == S[K:]))
    d_i = (child != S[:K]).sum(1)
    d_j = (child != S[K:]).sum(1)
    q = nv / (beta * Dij)  # probability of taking S_j where the parents differ
    sd = np.sqrt(Dij * q * (1 - q) / K)
    assert abs(d_i.mean() - nv / beta) < 4 * sd
    assert abs(d_j.mean() - (Dij - nv / beta)) < 4 * sd
    # beta * D <= |V|: the child is a copy of the second parent (clamped p_ij)
    c2 = oracle_mod.aux(42, 3, S[:2], np.array([1, 0], np.int32), np.array([20, 20], np.int32),
                        beta, 1)
    np.testing.assert_array_equal(c2[0], S[1])


def test_aux_variants_ux_and_no_crossover(oracle_mod):
    """Section 5.2: without crossover the offspring is its first parent; UX
    (p_ij = 1/2, Section 3.5.2) takes each differing position from either
    parent with probability 1/2, whatever D_ij and beta are."""
    rng = np.random.default_rng(1)
    nv, K = 300, 400
    S = rng.integers(1, 9, size=(2 * K, nv), dtype=np.uint8)
    partner = np.concatenate([np.arange(K, 2 * K), np.arange(K)]).astype(np.int32)
    dpart = rng.integers(1, nv, size=2 * K).astype(np.int32)
    none = oracle_mod.aux(7, 2, S, partner, dpart, 20, 1, mode=oracle_mod.X_NONE)
    np.testing.assert_array_equal(none, S)
    ux = oracle_mod.aux(7, 2, S, partner, dpart, 20, 1, mode=oracle_mod.X_UX)[:K]
    ux2 = oracle_mod.aux(7, 2, S, partner, np.full(2 * K, 5, np.int32), 3, 1,
                         mode=oracle_mod.X_UX)[:K]
    np.testing.assert_array_equal(ux, ux2)  # independent of D_ij and beta
    assert np.all((ux == S[:K]) | (ux == S[K:]))
    diff = S[:K] != S[K:]
    took_i = (ux == S[:K]) & diff
    n_diff = int(diff.sum())
    frac = took_i.sum() / n_diff
    assert abs(frac - 0.5) < 4 * np.sqrt(0.25 / n_diff)


def test_random_matching_is_uniform_over_the_others(oracle_mod):
    """Section 5.3: the second parent is any other individual, uniformly; it
    does not depend on the distances, and D_ij is reported for it."""
    p, G = 6, 3000
    rng = np.random.default_rng(2)
    D = rng.integers(0, 50, size=(p, p)).astype(np.int32)
    D2 = rng.integers(0, 50, size=(p, p)).astype(np.int32)
    uid = np.arange(p, dtype=np.uint64)
    counts = np.zeros((p, p))
    for g in range(1, G + 1):
        hist = np.zeros((p, 64), dtype=np.uint64)
        hc = np.zeros(p, dtype=np.int32)
        partner, dpart, _, _ = oracle_mod.match(D, uid, hist, hc, mode=oracle_mod.M_RANDOM,
                                                seed=99, gen=g)
        if g <= 20:
            other, _, _, _ = oracle_mod.match(D2, uid, hist, hc, mode=oracle_mod.M_RANDOM,
                                              seed=99, gen=g)
            np.testing.assert_array_equal(partner, other)
            np.testing.assert_array_equal(dpart, D[np.arange(p), partner])
        assert np.all(partner != np.arange(p))
        counts[np.arange(p), partner] += 1
    expect = G / (p - 1)
    off = ~np.eye(p, dtype=bool)
    assert np.all(np.abs(counts[off] - expect) < 5 * np.sqrt(expect))


def test_run_variants_stay_legal(oracle_mod):
    w = gen.workload_small()
    I = oracle_mod.Instance(w["grid"])
    for xo, mt, va in ((oracle_mod.X_UX, oracle_mod.M_NEAREST, 0),
                       (oracle_mod.X_NONE, oracle_mod.M_NEAREST, 0),
                       (oracle_mod.X_AUX, oracle_mod.M_RANDOM, 0),
                       (oracle_mod.X_AUX, oracle_mod.M_NEAREST, oracle_mod.V_PARTIAL)):
        r = I.run(I.params(depth=w["depth"], crossover=xo, matching=mt, variant=va), 16, 3,
                  w["seed"])
        assert r["filled"] <= I.ub
        assert gen.is_partial_latin(r["grid"])


# --- whole run (Alg. 2) ---------------------------------------------------------------------
def test_run_small_planted_reaches_optimum(oracle_mod):
    w = gen.workload_small()
    I = oracle_mod.Instance(w["grid"])
    r = I.run(I.params(depth=w["depth"]), w["population"], w["generations"], w["seed"])
    assert r["filled"] == 100 == I.ub
    g = r["grid"]
    assert gen.is_partial_latin(g)
    pre = w["grid"] != 0
    assert np.all(g[pre] == w["grid"][pre])
    assert np.all(np.diff(r["best_f"]) <= 0)


@pytest.mark.parametrize("seed", range(6))
def test_run_tiny_reaches_bruteforce_optimum(oracle_mod, seed):
    n = 4 + seed % 2
    g = gen.random_greedy(n, 0.4 + 0.1 * (seed % 3), 900 + seed)
    I = oracle_mod.Instance(g)
    r = I.run(I.params(depth=10 * n * n), 16, 5, 5000 + seed)
    opt = R.brute_force_optimum(g.tolist())
    assert r["filled"] <= I.ub
    assert r["filled"] == opt
    assert gen.is_partial_latin(r["grid"])


def test_run_stop_at_ub_and_determinism(oracle_mod):
    w = gen.workload_small()
    I = oracle_mod.Instance(w["grid"])
    P = I.params(depth=w["depth"], stop_at_ub=True)
    r1 = I.run(P, 32, 10, w["seed"])
    r2 = I.run(P, 32, 10, w["seed"])
    assert r1["gens"] == 1 and r1["filled"] == 100
    assert np.array_equal(r1["counters"], r2["counters"])
    assert np.array_equal(r1["grid"], r2["grid"])


# --- iteration budget (Section 4.3) --------------------------------------------------------
def test_run_iteration_cap_on_a_hard_instance(oracle_mod):
    """On an instance whose bound is out of reach no individual ends a phase
    early, so each generation runs exactly p * depth iterations and a cap C
    stops the run after generation ceil(C / (p * depth)); the capped run is the
    run with that many generations."""
    g = gen.random_greedy(12, 0.6, 5)
    I = oracle_mod.Instance(g)
    p, depth, G, seed = 8, 1440, 6, 77
    full = I.run(I.params(depth=depth), p, G, seed)
    assert full["filled"] < I.ub
    assert np.all(full["counters"][:, 0] == p * depth)
    per = p * depth
    for cap, stop in ((1, 1), (per, 1), (per + 1, 2), (3 * per - 1, 3), (3 * per, 3),
                      (G * per + 5, G)):
        r = I.run(I.params(depth=depth, max_iterations=cap), p, G, seed)
        assert r["gens"] == stop, (cap, r["gens"])
        short = I.run(I.params(depth=depth), p, stop, seed)
        assert r["filled"] == short["filled"]
        np.testing.assert_array_equal(r["grid"], short["grid"])
        np.testing.assert_array_equal(r["best_f"][:stop], full["best_f"][:stop])
        np.testing.assert_array_equal(r["counters"][:stop], full["counters"][:stop])
        assert np.all(r["counters"][stop:] == 0)


def test_run_iteration_cap_with_varying_generation_counts(oracle_mod):
    """Where individuals finish early the per-generation counts vary; the run
    stops at the first generation whose cumulative count reaches the cap."""
    g = gen.random_greedy(20, 0.5, 7)
    I = oracle_mod.Instance(g)
    p, depth, G, seed = 8, 4000, 6, 77
    full = I.run(I.params(depth=depth), p, G, seed)
    cum = np.cumsum(full["counters"][:, 0].astype(np.int64))
    assert len(set(full["counters"][:, 0].tolist())) > 1
    for k in range(G):
        for cap in (int(cum[k]), int(cum[k]) - 1):
            if cap <= 0:
                continue
            r = I.run(I.params(depth=depth, max_iterations=cap), p, G, seed)
            stop = 1 + int(np.argmax(cum >= cap))
            assert r["gens"] == stop
            np.testing.assert_array_equal(r["counters"][:stop], full["counters"][:stop])
