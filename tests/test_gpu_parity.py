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
@pytest.mark.parametrize("name,p,depth,lpv,wpb", [
    ("planted10", 64, 1000, 0, 0),
    ("planted10", 64, 1000, 8, 4),
    ("greedy12_60", 37, 1440, 1, 1),
    ("greedy12_60", 37, 1440, 2, 2),
    ("greedy20_50", 65, 4000, 4, 4),
    ("greedy20_50", 65, 4000, 0, 0),
    ("planted33_45", 20, 10890, 0, 0),
    ("planted33_45", 20, 10890, 1, 1),
    ("greedy70_70", 9, 6000, 0, 0),
    ("greedy70_70", 9, 6000, 8, 2),
])
def test_plits_parity(torch_cuda, oracle_mod, name, p, depth, lpv, wpb):
    """S', f' and every per-individual counter equal the oracle's."""
    g = _instances()[name]
    _say(f"plits {name} p={p} depth={depth} lpv={lpv} wpb={wpb}")
    s = P.Solver(g, depth=depth, lanes_per_vertex=lpv, waves_per_block=wpb)
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


def test_plits_from_conflicting_start(torch_cuda, oracle_mod):
    """A random (illegal, partial) start exercises both neighbourhoods, the
    repair and long eligible lists."""
    g = gen.random_greedy(20, 0.5, 7)
    _say("plits random start greedy20_50")
    s = P.Solver(g, depth=3000)
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


@pytest.mark.parametrize("p,gen_no,seed", [(2, 1, 1), (64, 3, 5), (100, 7, 11), (300, 2, 13),
                                           (1024, 4, 17)])
def test_select_parity(torch_cuda, oracle_mod, p, gen_no, seed):
    g = gen.random_greedy(20, 0.5, 7)
    _say(f"select p={p}")
    s = P.Solver(g)
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


# --- whole runs -------------------------------------------------------------------------
@pytest.mark.parametrize("name,p,G,depth,stop", [
    ("planted10", 64, 20, 1000, 0),
    ("greedy12_60", 32, 6, 1440, 0),
    ("greedy20_50", 48, 4, 2000, 0),
    ("planted10", 16, 8, 300, 1),
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
    for lpv, wpb in ((0, 0), (1, 1), (2, 2), (8, 4)):
        s = P.Solver(g, depth=2000, lanes_per_vertex=lpv, waves_per_block=wpb)
        for _ in range(2 if lpv == 0 and wpb == 0 else 1):
            grid, filled = s.solve(40, 3, 99)
            outs.append((grid.tobytes(), filled, s.stats()["totals"].tobytes()))
    assert len(set(outs)) == 1


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
