"""GPU path (libplse, gfx950) against the CPU oracle, stage by stage and whole
runs.  Every comparison is exact: all arithmetic is integer and both sides
draw the same counter-based random numbers, so the trajectories must agree
bit for bit.  Sizes span several tiles and ragged tails; full-size cases
compare sampled individuals that the oracle recomputes one by one."""

import sys

import numpy as np
import pytest

from paper_2103_10453_amd import instances as gen
from paper_2103_10453_amd import plse as P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _np(t):
    return t.detach().cpu().numpy()


def _instances():
    return {
        "planted10": gen.planted(10, 0.4, 0),
        "greedy12_60": gen.random_greedy(12, 0.6, 5),
        "greedy20_50": gen.random_greedy(20, 0.5, 7),
        "planted33_45": gen.planted(33, 0.45, 9),
        "greedy70_70": gen.random_greedy(70, 0.7, 2070),
    }


# --- init ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,p", [("planted10", 64), ("greedy12_60", 37), ("greedy20_50", 130),
                                    ("planted33_45", 70)])
def test_init_parity(torch_cuda, oracle_mod, name, p):
    g = _instances()[name]
    _say(f"init {name} p={p}")
    s = P.Solver(g)
    S, f = s.stage_init(p, 12345)
    torch_cuda.cuda.synchronize()
    I = oracle_mod.Instance(g)
    So, fo = I.init(12345, p)
    np.testing.assert_array_equal(_np(S)[:, :I.nv], So)
    np.testing.assert_array_equal(_np(f), fo)
    assert not _np(S)[:, I.nv:].any()


# --- PLITS --------------------------------------------------------------------------
@pytest.mark.parametrize("name,p,depth,spl,wpb", [
    ("planted10", 64, 1000, 0, 0),
    ("planted10", 64, 1000, 8, 4),
    ("greedy12_60", 37, 1440, 2, 1),
    ("greedy12_60", 37, 1440, 4, 2),
    ("greedy20_50", 65, 4000, 4, 4),
    ("greedy20_50", 65, 4000, 0, 0),
    ("planted33_45", 20, 10890, 0, 0),
    ("planted33_45", 20, 10890, 2, 1),
    ("greedy70_70", 9, 6000, 0, 0),
    ("greedy70_70", 9, 6000, 8, 2),
])
@pytest.mark.parametrize("kernel", [1, 2])
def test_plits_parity(torch_cuda, oracle_mod, name, p, depth, spl, wpb, kernel):
    """S', f' and every per-individual counter equal the oracle's, with the
    tabu table in global memory (kernel 1) and in LDS (kernel 2)."""
    g = _instances()[name]
    _say(f"plits {name} p={p} depth={depth} spl={spl} wpb={wpb} kernel={kernel}")
    s = P.Solver(g, depth=depth, slots_per_lane=spl, waves_per_block=wpb, plits_kernel=kernel)
    assert s.get_param("plits_kernel") == kernel
    # resident waves per CU of the chosen launch shape: at least one, at most
    # the 32 wave slots of a CU
    assert 1 <= s.get_param("plits_waves_per_cu") <= 32
    seed, gen_no = 777 + p, 3
    S0, _ = s.stage_init(p, seed)
    S1, f1, c1 = s.stage_plits(S0, gen_no, seed)
    torch_cuda.cuda.synchronize()
    I = oracle_mod.Instance(g)
    So, _ = I.init(seed, p)
    Po = I.params(depth=depth)
    S1o, f1o, c1o = I.plits(Po, seed, gen_no, list(range(p)), So)
    np.testing.assert_array_equal(_np(S1)[:, :I.nv], S1o)
    np.testing.assert_array_equal(_np(f1), f1o)
    np.testing.assert_array_equal(_np(c1).astype(np.uint64), c1o)


@pytest.mark.parametrize("kernel", [1, 2])
def test_plits_from_conflicting_start(torch_cuda, oracle_mod, kernel):
    """A random (illegal, partial) start exercises both neighbourhoods, the
    repair and long eligible lists."""
    g = gen.random_greedy(20, 0.5, 7)
    _say(f"plits random start greedy20_50 kernel={kernel}")
    s = P.Solver(g, depth=3000, plits_kernel=kernel)
    I = oracle_mod.Instance(g)
    vr, vc, off, dom = I.tables()
    rng = np.random.default_rng(3)
    p = 24
    S0 = np.zeros((p, s.stride), dtype=np.uint8)
    for i in range(p):
        for v in range(I.nv):
            choices = [0] + list(dom[off[v]:off[v + 1]])
            S0[i, v] = choices[rng.integers(0, len(choices))]
    import torch
    S0t = torch.from_numpy(S0).cuda()
    for depth1, depth2 in ((2500, 500), (40, 3), (0, 0)):
        s.set_param("depth1", depth1)
        s.set_param("depth2", depth2)
        S1, f1, c1 = s.stage_plits(S0t, 2, 99)
        torch.cuda.synchronize()
        Po = I.params(depth=0)
        Po[0], Po[1] = depth1, depth2
        S1o, f1o, c1o = I.plits(Po, 99, 2, list(range(p)), S0[:, :I.nv])
        np.testing.assert_array_equal(_np(S1)[:, :I.nv], S1o)
        np.testing.assert_array_equal(_np(f1), f1o)
        np.testing.assert_array_equal(_np(c1).astype(np.uint64), c1o)


@pytest.mark.parametrize("kernel,spl", [(1, 0), (2, 2), (2, 4), (2, 8)])
def test_plits_long_tenures(torch_cuda, oracle_mod, kernel, spl):
    """Tenures far beyond 125 iterations (alpha = 3 on a random start of a
    599-vertex grid): the LDS kernel keeps such expiries in the global tabu
    area and brings them back at its 128-iteration rebases; more than 256
    eligible vertices at the start cover the staged batches."""
    g = gen.planted(33, 0.45, 9)
    _say(f"plits long tenures planted33_45 kernel={kernel} spl={spl}")
    s = P.Solver(g, depth=4000, plits_kernel=kernel, slots_per_lane=spl,
                 alpha_num=3, alpha_den=1)
    I = oracle_mod.Instance(g)
    vr, vc, off, dom = I.tables()
    rng = np.random.default_rng(11)
    p = 12
    S0 = np.zeros((p, s.stride), dtype=np.uint8)
    for i in range(p):
        for v in range(I.nv):
            choices = [0] + list(dom[off[v]:off[v + 1]])
            S0[i, v] = choices[rng.integers(0, len(choices))]
    import torch
    S1, f1, c1 = s.stage_plits(torch.from_numpy(S0).cuda(), 4, 321)
    torch.cuda.synchronize()
    Po = I.params(depth=4000)
    Po[oracle_mod.P_ALPHA_NUM], Po[oracle_mod.P_ALPHA_DEN] = 3, 1
    S1o, f1o, c1o = I.plits(Po, 321, 4, list(range(p)), S0[:, :I.nv])
    np.testing.assert_array_equal(_np(S1)[:, :I.nv], S1o)
    np.testing.assert_array_equal(_np(f1), f1o)
    np.testing.assert_array_equal(_np(c1).astype(np.uint64), c1o)


# --- Partial-MPMA (Section 3.7) --------------------------------------------------------
@pytest.mark.parametrize("name,p,depth,spl,random_start", [
    ("greedy12_60", 37, 1440, 0, True),
    ("greedy20_50", 65, 4000, 4, True),
    ("greedy20_50", 40, 4000, 2, False),
    ("greedy70_70", 9, 6000, 8, True),
    ("greedy30_80", 33, 9000, 0, True),
])
def test_partial_plits_parity(torch_cuda, oracle_mod, name, p, depth, spl, random_start):
    """Repair of the offspring, then PartialCol: S', f' and every counter equal
    the oracle's."""
    g = gen.random_greedy(30, 0.8, 11) if name == "greedy30_80" else _instances()[name]
    _say(f"partial plits {name} p={p} depth={depth} spl={spl} random={random_start}")
    s = P.Solver(g, depth=depth, slots_per_lane=spl, variant=1)
    I = oracle_mod.Instance(g)
    import torch
    seed = 313 + p
    if random_start:
        vr, vc, off, dom = I.tables()
        rng = np.random.default_rng(seed)
        S0 = np.zeros((p, s.stride), dtype=np.uint8)
        for i in range(p):
            for v in range(I.nv):
                choices = [0] + list(dom[off[v]:off[v + 1]])
                S0[i, v] = choices[rng.integers(0, len(choices))]
        S0t = torch.from_numpy(S0).cuda()
        S0o = S0[:, :I.nv]
    else:
        S0t, _ = s.stage_init(p, seed)
        S0o, _ = I.init(seed, p)
    S1, f1, c1 = s.stage_plits(S0t, 2, seed)
    torch.cuda.synchronize()
    S1o, f1o, c1o = I.plits(I.params(depth=depth, variant=oracle_mod.V_PARTIAL), seed, 2,
                            list(range(p)), S0o)
    np.testing.assert_array_equal(_np(S1)[:, :I.nv], S1o)
    np.testing.assert_array_equal(_np(f1), f1o)
    np.testing.assert_array_equal(_np(c1).astype(np.uint64), c1o)


def test_partial_solve_parity(torch_cuda, oracle_mod):
    """A whole Partial-MPMA run (Section 3.7) equals the oracle's."""
    g = gen.random_greedy(25, 0.75, 3)
    _say("partial solve greedy25_75 p=32 G=4")
    s = P.Solver(g, depth=2500, variant=1)
    grid, filled = s.solve(32, 4, 55)
    st = s.stats()
    I = oracle_mod.Instance(g)
    r = I.run(I.params(depth=2500, variant=oracle_mod.V_PARTIAL), 32, 4, 55)
    assert filled == r["filled"]
    np.testing.assert_array_equal(grid, r["grid"])
    np.testing.assert_array_equal(st["counters_per_gen"], r["counters"][:r["gens"]])
    assert gen.is_partial_latin(grid)


# --- distances, selection, matching, crossover --------------------------------------
@pytest.mark.parametrize("name,m", [("planted10", 1), ("planted10", 130), ("greedy20_50", 200),
                                    ("planted33_45", 257), ("greedy70_70", 65)])
def test_distances_parity(torch_cuda, oracle_mod, name, m):
    g = _instances()[name]
    _say(f"distances {name} m={m}")
    s = P.Solver(g)
    I = oracle_mod.Instance(g)
    rng = np.random.default_rng(m)
    S = np.zeros((m, s.stride), dtype=np.uint8)
    S[:, :I.nv] = rng.integers(0, I.n + 1, size=(m, I.nv))
    for t in range(m // 4):  # some near-duplicates
        a, b = rng.integers(0, m, size=2)
        S[b] = S[a]
    import torch
    D = s.stage_distances(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    Do = oracle_mod.distances(S[:, :I.nv], S[:, :I.nv])
    np.testing.assert_array_equal(_np(D).astype(np.int32), Do)


@pytest.mark.parametrize("p,gen_no,seed,global_sort", [(2, 1, 1, 0), (64, 3, 5, 0),
                                                       (100, 7, 11, 0), (300, 2, 13, 0),
                                                       (1024, 4, 17, 0), (2100, 5, 19, 1),
                                                       (4097, 6, 23, 1)])
def test_select_parity(torch_cuda, oracle_mod, p, gen_no, seed, global_sort):
    """Alg. 4 on the GPU equals the oracle; global_sort exercises the key
    sort used when the keys exceed LDS (tiles plus global merge steps)."""
    g = gen.random_greedy(20, 0.5, 7)
    _say(f"select p={p} global_sort={global_sort}")
    s = P.Solver(g, select_global_sort=global_sort)
    I = oracle_mod.Instance(g)
    rng = np.random.default_rng(seed)
    m = 2 * p
    X = rng.integers(0, 3, size=(m, I.nv), dtype=np.uint8)
    for t in range(m // 3):
        a, b = rng.integers(0, m, size=2)
        X[b] = X[a]
        X[b, rng.integers(0, I.nv, size=rng.integers(0, I.nv // 6 + 1))] = 1
    # one candidate close to many (exceeds the close-list capacity)
    for t in range(min(m, 60)):
        X[t] = X[0]
        X[t, rng.integers(0, I.nv, size=3)] = 2
    Do = oracle_mod.distances(X, X)
    f = rng.integers(0, 4, size=m).astype(np.int32)
    import torch
    acc = s.stage_select(torch.from_numpy(f).cuda(), torch.from_numpy(Do.astype(np.int16)).cuda(),
                         gen_no, seed)
    torch.cuda.synchronize()
    acc_o = oracle_mod.select(I.nv, p, 10, seed, gen_no, f, Do)
    np.testing.assert_array_equal(_np(acc), acc_o)


@pytest.mark.parametrize("p,seed", [(2, 1), (24, 2), (130, 3), (513, 4)])
def test_match_parity(torch_cuda, oracle_mod, p, seed):
    _say(f"match p={p}")
    g = gen.planted(10, 0.4, 0)
    s = P.Solver(g)
    rng = np.random.default_rng(seed)
    D = rng.integers(0, 9, size=(p, p)).astype(np.int32)
    D = np.minimum(D, D.T)
    uid = (rng.permutation(10 * p)[:p] + (5 << 32)).astype(np.uint64)
    hist = np.zeros((p, 64), dtype=np.uint64)
    hc = np.zeros(p, dtype=np.int32)
    for i in range(p):
        k = int(rng.integers(0, 90))
        pool = np.concatenate([uid, (rng.integers(0, 10 * p, size=8) + (9 << 32)).astype(np.uint64)])
        ex = rng.choice(pool, size=min(k, 64, len(pool)), replace=False)
        hist[i, :len(ex)] = ex
        hc[i] = k if (k >= 64 and len(ex) == 64) else len(ex)
    import torch
    hist_t = torch.from_numpy(hist.view(np.int64)).cuda()
    hc_t = torch.from_numpy(hc).cuda()
    partner, dpart = s.stage_match(torch.from_numpy(D.astype(np.int16)).cuda(),
                                   torch.from_numpy(uid.view(np.int64)).cuda(), hist_t, hc_t)
    torch.cuda.synchronize()
    po, do, ho, hco = oracle_mod.match(D, uid, hist, hc)
    np.testing.assert_array_equal(_np(partner), po)
    np.testing.assert_array_equal(_np(dpart), do)
    np.testing.assert_array_equal(_np(hist_t).view(np.uint64), ho)
    np.testing.assert_array_equal(_np(hc_t), hco)


@pytest.mark.parametrize("name,p,seed", [("planted10", 64, 3), ("greedy20_50", 33, 4),
                                         ("greedy70_70", 17, 5)])
def test_aux_parity(torch_cuda, oracle_mod, name, p, seed):
    g = _instances()[name]
    _say(f"aux {name} p={p}")
    s = P.Solver(g)
    I = oracle_mod.Instance(g)
    rng = np.random.default_rng(seed)
    S = np.zeros((p, s.stride), dtype=np.uint8)
    S[:, :I.nv] = rng.integers(0, I.n + 1, size=(p, I.nv))
    partner = np.array([(i + 1 + rng.integers(0, p - 1)) % p for i in range(p)], dtype=np.int32)
    dpart = rng.integers(0, I.nv + 1, size=p).astype(np.int32)
    dpart[0] = 0
    import torch
    out = s.stage_aux(torch.from_numpy(S).cuda(), torch.from_numpy(partner).cuda(),
                      torch.from_numpy(dpart).cuda(), 6, seed)
    torch.cuda.synchronize()
    oo = oracle_mod.aux(seed, 6, S[:, :I.nv], partner, dpart)
    np.testing.assert_array_equal(_np(out)[:, :I.nv], oo)


@pytest.mark.parametrize("mode", [1, 2])
def test_aux_variant_parity(torch_cuda, oracle_mod, mode):
    """UX (1) and no crossover (2), Section 3.5.2 and Section 5.2."""
    g = _instances()["greedy20_50"]
    _say(f"aux variant {mode}")
    s = P.Solver(g, crossover=mode)
    I = oracle_mod.Instance(g)
    p, seed = 40, 8
    rng = np.random.default_rng(seed)
    S = np.zeros((p, s.stride), dtype=np.uint8)
    S[:, :I.nv] = rng.integers(0, I.n + 1, size=(p, I.nv))
    partner = np.array([(i + 1 + rng.integers(0, p - 1)) % p for i in range(p)], dtype=np.int32)
    dpart = rng.integers(0, I.nv + 1, size=p).astype(np.int32)
    import torch
    out = s.stage_aux(torch.from_numpy(S).cuda(), torch.from_numpy(partner).cuda(),
                      torch.from_numpy(dpart).cuda(), 3, seed)
    torch.cuda.synchronize()
    oo = oracle_mod.aux(seed, 3, S[:, :I.nv], partner, dpart, mode=mode)
    np.testing.assert_array_equal(_np(out)[:, :I.nv], oo)


# --- whole runs -------------------------------------------------------------------------
@pytest.mark.parametrize("name,p,G,depth,crossover,matching", [
    ("planted10", 32, 6, 600, 1, 0),
    ("greedy12_60", 24, 5, 1440, 2, 0),
    ("greedy20_50", 32, 4, 2000, 0, 1),
    ("greedy12_60", 24, 5, 1440, 1, 1),
])
def test_solve_variant_parity(torch_cuda, oracle_mod, name, p, G, depth, crossover, matching):
    """Whole runs with the crossover / matching variants of Sections 5.2-5.3."""
    g = _instances()[name]
    _say(f"solve variant {name} p={p} G={G} crossover={crossover} matching={matching}")
    s = P.Solver(g, depth=depth, crossover=crossover, matching=matching)
    seed = 777 + p
    grid, filled = s.solve(p, G, seed)
    st = s.stats()
    I = oracle_mod.Instance(g)
    r = I.run(I.params(depth=depth, crossover=crossover, matching=matching), p, G, seed)
    assert filled == r["filled"]
    np.testing.assert_array_equal(grid, r["grid"])
    np.testing.assert_array_equal(st["best_f_per_gen"], r["best_f"][:r["gens"]])
    np.testing.assert_array_equal(st["counters_per_gen"], r["counters"][:r["gens"]])


@pytest.mark.parametrize("name,p,G,depth,stop", [
    ("planted10", 64, 20, 1000, 0),
    ("greedy12_60", 32, 6, 1440, 0),
    ("greedy20_50", 48, 4, 2000, 0),
    ("planted10", 16, 8, 300, 1),
    # populations not a multiple of 4: 2p % 8 != 0 takes the one-entry-per-lane
    # scans of close lists and matching
    ("greedy12_60", 30, 4, 1440, 0),
    ("planted10", 18, 5, 600, 0),
])
def test_solve_parity(torch_cuda, oracle_mod, name, p, G, depth, stop):
    g = _instances()[name]
    _say(f"solve {name} p={p} G={G} depth={depth} stop={stop}")
    s = P.Solver(g, depth=depth, stop_at_ub=stop)
    seed = 4242 + p
    grid, filled = s.solve(p, G, seed)
    st = s.stats()
    I = oracle_mod.Instance(g)
    r = I.run(I.params(depth=depth, stop_at_ub=bool(stop)), p, G, seed)
    assert filled == r["filled"]
    np.testing.assert_array_equal(grid, r["grid"])
    assert st["generations_run"] == r["gens"]
    np.testing.assert_array_equal(st["best_f_per_gen"], r["best_f"][:r["gens"]])
    np.testing.assert_array_equal(st["counters_per_gen"], r["counters"][:r["gens"]])
    assert filled <= s.ub and gen.is_partial_latin(grid)


def test_solve_repeatable_and_shape_independent(torch_cuda):
    """Same result on a second call and under other launch shapes / table types."""
    g = gen.random_greedy(20, 0.5, 7)
    _say("solve repeat")
    outs = []
    for spl, wpb in ((0, 0), (2, 1), (4, 2), (8, 4)):
        s = P.Solver(g, depth=2000, slots_per_lane=spl, waves_per_block=wpb)
        for _ in range(2 if spl == 0 and wpb == 0 else 1):
            grid, filled = s.solve(40, 3, 99)
            outs.append((grid.tobytes(), filled, s.stats()["totals"].tobytes()))
    assert len(set(outs)) == 1


@pytest.mark.parametrize("p", [40, 200])
def test_stage_timing_keeps_results(torch_cuda, p):
    """The stage-timed mode (stages one by one between events, distances among
    P_t before the search) gives the graph-replay result, with a positive time
    for every stage of every generation (p >= 64: distances among P_t are a
    stage of their own)."""
    g = gen.random_greedy(20, 0.5, 7)
    _say(f"stage timing p={p}")
    s = P.Solver(g, depth=2000)
    ref = s.solve(p, 3, 5)
    ref_tot = s.stats()["totals"].copy()
    assert s.stage_timing().shape == (0, len(P.STAGES))
    s.set_param("stage_timing", 1)
    grid, filled = s.solve(p, 3, 5)
    assert filled == ref[1] and np.array_equal(grid, ref[0])
    assert np.array_equal(s.stats()["totals"], ref_tot)
    st = s.stage_timing()
    assert st.shape == (3, len(P.STAGES))
    cols = [i for i, name in enumerate(P.STAGES) if p >= 64 or name != "distances_Pt"]
    assert (st[:, cols] > 0).all()
    ms_plits, _ = s.timing()
    np.testing.assert_allclose(st[:, 1], ms_plits, rtol=0.25, atol=0.05)


# --- full size: sampled individuals --------------------------------------------------
def test_full_size_n50_generation_sampled(torch_cuda, oracle_mod):
    """Planted n=50, 50% prefilled, population 16384, depth 10 n^2 as timed by
    the benchmark: init and generation-1 PLITS of the whole population on the
    GPU, compared on sampled slots recomputed one by one by the oracle."""
    w = gen.workload_n50()
    _say("full-size n50 p=16384 init+plits sampled")
    s = P.Solver(w["grid"], depth=w["depth"])
    p = w["population"]
    S0, f0 = s.stage_init(p, w["seed"])
    S1, f1, c1 = s.stage_plits(S0, 1, w["seed"])
    torch_cuda.cuda.synchronize()
    I = oracle_mod.Instance(w["grid"])
    slots = [0, 1, 63, 64, 4097, 8191, 12000, p - 1]
    So, fo = I.init_slots(w["seed"], slots)
    np.testing.assert_array_equal(_np(S0)[slots, :I.nv], So)
    np.testing.assert_array_equal(_np(f0)[slots], fo)
    S1o, f1o, c1o = I.plits(I.params(depth=w["depth"]), w["seed"], 1, slots, So)
    np.testing.assert_array_equal(_np(S1)[slots, :I.nv], S1o)
    np.testing.assert_array_equal(_np(f1)[slots], f1o)
    np.testing.assert_array_equal(_np(c1)[slots].astype(np.uint64), c1o)
    # every output is a legal colouring within the domains
    Sfull = _np(S1)[:, :I.nv]
    assert Sfull.max() <= I.n


# --- batched solve ---------------------------------------------------------------------
@pytest.mark.parametrize("persistent", [1, 0])
def test_batch_equals_standalone_and_oracle(torch_cuda, oracle_mod, persistent):
    """plse_solve_batch over instances of different orders returns, for each,
    exactly what plse_solve returns alone and what the oracle computes, with
    the searches as persistent launches over (instance, individual) items and
    as a grid per instance."""
    names = ["greedy20_50", "planted10", "greedy12_60", "planted33_45", "greedy70_70",
             "planted10"]
    grids = [_instances()[k] for k in names]
    _say(f"batch of 6 mixed instances p=32 G=4 persistent={persistent}")
    p, G = 32, 4
    seeds = [11 + 7 * i for i in range(len(grids))]
    solvers = [P.Solver(g, depth=int(10 * g.shape[0] ** 2 // 4), persistent=persistent)
               for g in grids]
    res = P.Solver.solve_batch(solvers, p, G, seeds)
    batch_stats = [s.stats() for s in solvers]
    for i, g in enumerate(grids):
        alone = P.Solver(g, depth=int(10 * g.shape[0] ** 2 // 4))
        grid, filled = alone.solve(p, G, seeds[i])
        assert filled == res[i][1]
        np.testing.assert_array_equal(grid, res[i][0])
        np.testing.assert_array_equal(alone.stats()["counters_per_gen"],
                                      batch_stats[i]["counters_per_gen"])
        I = oracle_mod.Instance(g)
        r = I.run(I.params(depth=int(10 * g.shape[0] ** 2 // 4)), p, G, seeds[i])
        assert r["filled"] == res[i][1]
        np.testing.assert_array_equal(r["grid"], res[i][0])
        np.testing.assert_array_equal(r["counters"], batch_stats[i]["counters_per_gen"])


def test_batch_mixed_searches_equal_standalone(torch_cuda, oracle_mod):
    """A batch whose instances need different search launches (Partial-MPMA,
    the LDS-resident kernel, MPMA at two chunk sizes) forms several launch
    groups, captured as branches of one graph per generation; each instance
    still returns exactly what it returns alone, and the oracle's result."""
    specs = [("greedy20_50", dict(variant=1)), ("planted33_45", dict(variant=1)),
             ("greedy12_60", dict(plits_kernel=2)), ("greedy20_50", dict(slots_per_lane=4)),
             ("planted10", dict()), ("greedy70_70", dict())]
    _say("batch of 6 instances with different search launches p=24 G=3")
    p, G = 24, 3
    seeds = [31 + 5 * i for i in range(len(specs))]
    depth = lambda g: int(10 * g.shape[0] ** 2 // 4)
    grids = [_instances()[k] for k, _ in specs]
    solvers = [P.Solver(g, depth=depth(g), **kw) for g, (_, kw) in zip(grids, specs)]
    res = P.Solver.solve_batch(solvers, p, G, seeds)
    for i, (g, (name, kw)) in enumerate(zip(grids, specs)):
        alone = P.Solver(g, depth=depth(g), **kw)
        grid, filled = alone.solve(p, G, seeds[i])
        assert filled == res[i][1], name
        np.testing.assert_array_equal(grid, res[i][0])
    I = oracle_mod.Instance(grids[0])
    r = I.run(I.params(depth=depth(grids[0]), variant=oracle_mod.V_PARTIAL), p, G, seeds[0])
    assert r["filled"] == res[0][1]
    np.testing.assert_array_equal(r["grid"], res[0][0])


def test_batch_session_steps_in_parts(torch_cuda):
    """plse_batch_begin / step / step / end equals plse_solve_batch in one go."""
    names = ["greedy20_50", "planted10", "planted33_45"]
    grids = [_instances()[k] for k in names]
    _say("batch session in parts")
    p, seeds = 24, [5, 6, 7]
    solvers = [P.Solver(g, depth=800) for g in grids]
    ref = P.Solver.solve_batch(solvers, p, 3, seeds)
    ref_cnt = [s.stats()["counters_per_gen"].copy() for s in solvers]
    b = P.plse_batch_begin([s.h for s in solvers], p, seeds)
    P.plse_batch_step(b, 2)
    P.plse_batch_step(b, 1)
    got = P.plse_batch_end(b, [g.shape[0] for g in grids])
    for (g1, f1), (g2, f2), s, c in zip(ref, got, solvers, ref_cnt):
        assert f1 == f2 and np.array_equal(g1, g2)
        np.testing.assert_array_equal(s.stats()["counters_per_gen"], c)
    # the handles are free again
    solvers[0].solve(p, 1, 1)


def test_batch_more_than_one_launch_chunk(torch_cuda, oracle_mod):
    """More instances than one launch list holds (130 > 128), tiny sizes."""
    _say("batch of 130 tiny instances p=8 G=2")
    grids = [gen.random_greedy(4 + i % 5, 0.3 + 0.05 * (i % 5), 5000 + i) for i in range(130)]
    solvers = [P.Solver(g, depth=60) for g in grids]
    seeds = [900 + i for i in range(130)]
    res = P.Solver.solve_batch(solvers, 8, 2, seeds)
    for i in (0, 1, 63, 127, 128, 129):
        I = oracle_mod.Instance(grids[i])
        r = I.run(I.params(depth=60), 8, 2, seeds[i])
        assert r["filled"] == res[i][1]
        np.testing.assert_array_equal(r["grid"], res[i][0])


# --- serving -------------------------------------------------------------------------------
def _wait(srv, tickets, timeout_s=120.0):
    import time
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout_s, "server did not finish in time"
        time.sleep(0.002)
    return out


def test_served_results_equal_alone_and_in_mix(torch_cuda):
    """Each request served alone and inside a mix of requests that arrive while
    others run returns exactly what plse_solve returns (continuous batching)."""
    import time
    _say("serving: alone vs mix")
    specs = [(gen.random_greedy(20, 0.5, 7), 24, 3, 1), (gen.planted(10, 0.4, 0), 16, 5, 2),
             (gen.random_greedy(12, 0.6, 5), 24, 4, 3), (gen.planted(33, 0.45, 9), 16, 2, 4),
             (gen.random_greedy(15, 0.4, 21), 24, 3, 5)]
    want = []
    for g, p, G, seed in specs:
        s = P.Solver(g, depth=300)
        want.append(s.solve(p, G, seed))
    srv = P.Server(1 << 30, max_slots=3)
    try:
        # alone, one after the other
        for i, (g, p, G, seed) in enumerate(specs):
            t = srv.submit(P.Solver(g, depth=300), p, G, seed)
            r = _wait(srv, [t])[t]
            assert r["status"] == P.PLSE_OK and r["generations"] == G
            assert r["filled"] == want[i][1]
            np.testing.assert_array_equal(r["grid"], want[i][0])
        # mixed: staggered arrivals, at most three resident at once
        tickets = []
        for i, (g, p, G, seed) in enumerate(specs):
            tickets.append(srv.submit(P.Solver(g, depth=300), p, G, seed))
            time.sleep(0.003 * i)
        res = _wait(srv, tickets)
        for i, t in enumerate(tickets):
            assert res[t]["status"] == P.PLSE_OK
            assert res[t]["filled"] == want[i][1]
            np.testing.assert_array_equal(res[t]["grid"], want[i][0])
            assert res[t]["admit_s"] >= res[t]["submit_s"] and res[t]["done_s"] >= res[t]["admit_s"]
    finally:
        srv.close()


def test_served_variants_equal_alone(torch_cuda):
    """Requests with Partial-MPMA, the LDS-resident search kernel, the UX
    crossover and random matching, served together, each return what
    plse_solve returns for them alone."""
    _say("serving: variants in one mix")
    specs = [(gen.random_greedy(20, 0.5, 7), dict(variant=1)),
             (gen.planted(33, 0.45, 9), dict(plits_kernel=2)),
             (gen.random_greedy(12, 0.6, 5), dict(crossover=1, matching=1)),
             (gen.random_greedy(15, 0.4, 21), dict(slots_per_lane=2, waves_per_block=2))]
    p, G = 16, 3
    want = [P.Solver(g, depth=300, **kw).solve(p, G, 40 + i) for i, (g, kw) in enumerate(specs)]
    srv = P.Server(1 << 30, max_slots=4)
    try:
        tickets = [srv.submit(P.Solver(g, depth=300, **kw), p, G, 40 + i)
                   for i, (g, kw) in enumerate(specs)]
        res = _wait(srv, tickets)
        for i, t in enumerate(tickets):
            assert res[t]["status"] == P.PLSE_OK
            assert res[t]["filled"] == want[i][1]
            np.testing.assert_array_equal(res[t]["grid"], want[i][0])
    finally:
        srv.close()


def test_server_capacity_and_fault_isolation(torch_cuda):
    _say("serving: capacity refusal and fault hook")
    small = P.Solver(gen.planted(10, 0.4, 0), depth=200)
    big = P.Solver(gen.random_greedy(40, 0.3, 3), depth=200)
    budget = small.ensure_workspace(16).numel() * 3
    srv = P.Server(budget, max_slots=4)
    try:
        with pytest.raises(P.PlseError) as e:
            srv.submit(big, 2048, 2, 1)
        assert e.value.status == P.PLSE_E_CAPACITY
        a = P.Solver(gen.planted(10, 0.4, 0), depth=200)
        b = P.Solver(gen.planted(10, 0.4, 0), depth=200, fail_at_generation=2)
        c = P.Solver(gen.random_greedy(12, 0.6, 5), depth=200)
        ta, tb, tc = srv.submit(a, 16, 4, 7), srv.submit(b, 16, 4, 8), srv.submit(c, 16, 4, 9)
        res = _wait(srv, [ta, tb, tc])
        assert res[tb]["status"] == P.PLSE_E_FAULT and res[tb]["generations"] == 2
        for solver, t, seed in ((a, ta, 7), (c, tc, 9)):
            ref = P.Solver(solver.grid, depth=200).solve(16, 4, seed)
            assert res[t]["status"] == P.PLSE_OK and res[t]["filled"] == ref[1]
            np.testing.assert_array_equal(res[t]["grid"], ref[0])
    finally:
        srv.close()


# --- degenerate and extreme instances ----------------------------------------------------
def _edge_instances():
    return {
        "full10": gen.planted(10, 1.0, 0),                  # every cell prefilled: no vertex
        "n1_empty": np.zeros((1, 1), dtype=np.int8),        # smallest order
        "n2_empty": np.zeros((2, 2), dtype=np.int8),
        "empty12": np.zeros((12, 12), dtype=np.int8),       # no prefilled cell: full domains
        "greedy100_30": gen.random_greedy(100, 0.3, 4),     # order 100, 30 % prefilled
        "planted127_60": gen.planted(127, 0.6, 1),          # largest order the boundary accepts
        "greedy127_50": gen.random_greedy(127, 0.5, 1),
    }


@pytest.mark.parametrize("name,p,G,depth", [
    ("full10", 4, 2, 100), ("n1_empty", 2, 2, 10), ("n2_empty", 4, 3, 40),
    ("empty12", 16, 3, 1440), ("greedy100_30", 4, 2, 3000), ("planted127_60", 4, 2, 3000),
    ("greedy127_50", 6, 2, 3000),
])
def test_solve_degenerate_and_extreme_orders(torch_cuda, oracle_mod, name, p, G, depth):
    """Whole runs on an instance without vertices, the smallest orders, an
    empty grid, and orders 100 and 127 (7 colour bit planes, 128 colours per
    row of counts) equal the oracle's."""
    g = _edge_instances()[name]
    _say(f"solve edge {name} p={p} G={G} depth={depth}")
    s = P.Solver(g, depth=depth)
    grid, filled = s.solve(p, G, 31 + p)
    st = s.stats()
    I = oracle_mod.Instance(g)
    r = I.run(I.params(depth=depth), p, G, 31 + p)
    assert filled == r["filled"] and st["generations_run"] == r["gens"]
    np.testing.assert_array_equal(grid, r["grid"])
    np.testing.assert_array_equal(st["best_f_per_gen"], r["best_f"][:r["gens"]])
    np.testing.assert_array_equal(st["counters_per_gen"], r["counters"][:r["gens"]])
    assert filled <= s.ub and gen.is_partial_latin(grid)


# --- launch-shape autotuning ---------------------------------------------------------------
def test_autotune_keeps_the_fastest_fitting_shape_and_the_results(torch_cuda, oracle_mod):
    """plse_autotune times every chunk size that fits, keeps the fastest,
    and a solve under the chosen size (alone and in a batch with other
    autotuned instances) still equals the oracle."""
    names = ["greedy12_60", "greedy20_50", "planted33_45"]
    grids = [_instances()[k] for k in names]
    solvers = []
    for k, g in zip(names, grids):
        _say(f"autotune {k}")
        s = P.Solver(g, depth=600)
        ms = s.autotune(sample=48, depth=300, seed=3)
        fit = ms >= 0
        assert fit.any() and np.all(ms[fit] > 0)
        assert s.get_param("slots_per_lane") == (2, 4, 8)[int(np.argmin(np.where(fit, ms, np.inf)))]
        solvers.append(s)
    seeds = [71, 72, 73]
    res = P.Solver.solve_batch(solvers, 24, 3, seeds)
    for g, s, sd, (grid, filled) in zip(grids, solvers, seeds, res):
        I = oracle_mod.Instance(g)
        r = I.run(I.params(depth=600), 24, 3, sd)
        assert filled == r["filled"]
        np.testing.assert_array_equal(grid, r["grid"])
        grid2, filled2 = s.solve(24, 3, sd)
        assert filled2 == r["filled"]
        np.testing.assert_array_equal(grid2, r["grid"])


def test_autotune_shape_keeps_the_fastest_shape_and_the_results(torch_cuda, oracle_mod):
    """plse_autotune_shape times chunk size x waves per block, keeps the
    fastest pair, and a batch of instances tuned apart (different shapes in
    one persistent launch group) still equals the oracle."""
    names = ["greedy20_50", "planted33_45", "greedy12_60"]
    grids = [_instances()[k] for k in names]
    solvers = []
    for k, g in zip(names, grids):
        _say(f"autotune shape {k}")
        s = P.Solver(g, depth=600)
        ms = s.autotune_shape(sample=48, depth=300, seed=5)
        assert ms.shape == (3, 3)
        fit = ms >= 0
        assert fit.any() and np.all(ms[fit] > 0)
        w, c = np.unravel_index(int(np.argmin(np.where(fit, ms, np.inf))), ms.shape)
        assert s.get_param("waves_per_block") == (1, 2, 4)[w]
        assert s.get_param("slots_per_lane") == (2, 4, 8)[c]
        solvers.append(s)
    seeds = [81, 82, 83]
    res = P.Solver.solve_batch(solvers, 24, 3, seeds)
    for g, sd, (grid, filled) in zip(grids, seeds, res):
        I = oracle_mod.Instance(g)
        r = I.run(I.params(depth=600), 24, 3, sd)
        assert filled == r["filled"]
        np.testing.assert_array_equal(grid, r["grid"])


def test_c_example_solves_like_the_oracle(torch_cuda, oracle_mod):
    """The plain-C driver (its own process and HIP runtime, caller-owned
    workspace from hipMalloc) returns the oracle's grid."""
    import os
    import subprocess
    exe = os.path.join(os.path.dirname(P.library_path()), "examples", "plse_solve")
    if not os.path.exists(exe):
        pytest.skip("C example not built")
    g = _instances()["greedy12_60"]
    n = g.shape[0]
    _say("C example greedy12_60 p=24 G=3")
    text = f"{n}\n" + "\n".join(" ".join(str(int(v)) for v in row) for row in g) + "\n"
    r = subprocess.run([exe, "24", "3", "17", "1440"], input=text.encode(), capture_output=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr.decode()
    lines = r.stdout.decode().split("\n")
    head = lines[0].split()
    grid = np.array([[int(v) for v in lines[2 + i].split()] for i in range(n)], dtype=np.int8)
    I = oracle_mod.Instance(g)
    o = I.run(I.params(depth=1440), 24, 3, 17)
    assert int(head[1]) == o["filled"] and int(head[3]) == I.ub and int(head[5]) == o["gens"]
    np.testing.assert_array_equal(grid, o["grid"])


def test_select_full_size_parity(torch_cuda, oracle_mod):
    """Alg. 4 at the benchmark's full size (2p = 32768 candidates, keys sorted
    in global memory) equals the oracle; candidates fall in clusters of about
    five mutually close ones (D within the spacing), the rest far apart."""
    g = gen.random_greedy(20, 0.5, 7)
    s = P.Solver(g)
    I = oracle_mod.Instance(g)
    p = 16384
    m = 2 * p
    _say(f"select full size m={m}")
    rng = np.random.default_rng(5)
    cl = rng.integers(0, 6000, size=m)
    D = np.empty((m, m), dtype=np.int16)
    for r0 in range(0, m, 4096):
        D[r0:r0 + 4096] = np.where(cl[r0:r0 + 4096, None] == cl[None, :], np.int16(4),
                                   np.int16(90))
    np.fill_diagonal(D, 0)
    f = rng.integers(0, 40, size=m).astype(np.int32)
    import torch
    Dg = torch.from_numpy(D).cuda()
    for gen_no in (1, 7):
        acc = s.stage_select(torch.from_numpy(f).cuda(), Dg, gen_no, 11)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_np(acc), oracle_mod.select(I.nv, p, 10, 11, gen_no, f, D))


def test_generation_stages_full_size(torch_cuda, oracle_mod):
    """Distances, matching and AUX at the n=50 workload's full size (p = 16384,
    2p = 32768 rows of 1250 vertices): sampled rows of D recomputed by the
    oracle, and the whole matching and crossover of the population."""
    w = gen.workload_n50()
    g = w["grid"]
    s = P.Solver(g, depth=w["depth"])
    I = oracle_mod.Instance(g)
    p = 16384
    m = 2 * p
    _say(f"generation stages full size p={p}")
    rng = np.random.default_rng(8)
    S = np.zeros((m, s.stride), dtype=np.uint8)
    S[:, :I.nv] = rng.integers(0, I.n + 1, size=(m, I.nv), dtype=np.uint8)
    for t in range(2000):  # near copies, so that distances span the range
        a, b = rng.integers(0, m, size=2)
        S[b, :I.nv] = S[a, :I.nv]
        S[b, rng.integers(0, I.nv, size=int(rng.integers(0, 40)))] = 0
    import torch
    D = s.stage_distances(torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    rows = np.array([0, 1, 63, 64, 4097, 16383, 16384, 20000, 32767])
    Dr = _np(D[torch.from_numpy(rows).cuda()]).astype(np.int32)
    np.testing.assert_array_equal(Dr, oracle_mod.distances(S[rows, :I.nv], S[:, :I.nv]))
    # matching among the first p rows, empty histories
    Dp = D[:p, :p].contiguous()
    uid = (np.arange(p, dtype=np.uint64) + (3 << 32)).astype(np.uint64)
    hist = np.zeros((p, 64), dtype=np.uint64)
    hc = np.zeros(p, dtype=np.int32)
    hist_t = torch.from_numpy(hist.view(np.int64)).cuda()
    hc_t = torch.from_numpy(hc).cuda()
    partner, dpart = s.stage_match(Dp, torch.from_numpy(uid.view(np.int64)).cuda(), hist_t, hc_t)
    torch.cuda.synchronize()
    po, do, ho, hco = oracle_mod.match(_np(Dp).astype(np.int32), uid, hist, hc)
    np.testing.assert_array_equal(_np(partner), po)
    np.testing.assert_array_equal(_np(dpart), do)
    # AUX offspring of the whole population
    out = s.stage_aux(torch.from_numpy(S[:p]).cuda(), partner, dpart, 2, 77)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(out)[:, :I.nv], oracle_mod.aux(77, 2, S[:p, :I.nv], po, do))
