"""GPU path against the oracle at the benchmark's sizes.

- A whole run of the planted n = 50 grid (50 % prefilled) at population 256,
  three generations of full depth 10 n^2: the best grid, best f and every
  counter per generation, and the whole state of Alg. 2 after the run (the
  population, f, uids, partner histories, the offspring of the next
  generation, S*), read from a checkpoint image.
- Whole runs at the benchmark's population, 16384: the in-graph selection
  over 2p = 32768 candidates (keys sorted in global memory), the gather and
  the matching through the candidate-to-individual maps, AUX and the
  searches of later generations, on grids small enough for the oracle to
  recompute every distance of P_t u P'.
- Generation-1 searches of the 70x70 random-greedy grids at 30, 50 and 70 %
  prefilled with their full depth 49000 and population 16384, on sampled
  slots the oracle recomputes one by one.
"""

import struct
import sys

import numpy as np
import pytest

from paper_2103_10453_amd import instances as gen
from paper_2103_10453_amd import plse as P

pytestmark = pytest.mark.gpu

HIST = 64
CTL_BYTES = 32        # Ctl: six int32 and the cumulative iteration count
HEADER_BYTES = 48


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def parse_checkpoint(img, nv):
    """The regions of a checkpoint image (include/plse.h): header, control
    block, per-generation records, S*, P_t, f, uids, histories, their
    counts, the offspring."""
    b = bytes(np.asarray(img, dtype=np.uint8))
    magic, version, n, nv_, stride, p = struct.unpack_from("<IIiiii", b, 0)
    gens = struct.unpack_from("<i", b, 40)[0]
    assert nv_ == nv
    o = HEADER_BYTES + CTL_BYTES
    rec = 8 + 8 * P.NCOUNTERS
    stats = np.frombuffer(b, dtype=np.uint8, count=rec * gens, offset=o).reshape(gens, rec)
    o += rec * gens
    star = np.frombuffer(b, dtype=np.uint8, count=stride, offset=o)[:nv]
    o += stride
    S = np.frombuffer(b, dtype=np.uint8, count=p * stride, offset=o).reshape(p, stride)[:, :nv]
    o += p * stride
    f = np.frombuffer(b, dtype=np.int32, count=p, offset=o)
    o += 4 * p
    uid = np.frombuffer(b, dtype=np.uint64, count=p, offset=o)
    o += 8 * p
    hist = np.frombuffer(b, dtype=np.uint64, count=p * HIST, offset=o).reshape(p, HIST)
    o += 8 * p * HIST
    hc = np.frombuffer(b, dtype=np.int32, count=p, offset=o)
    o += 4 * p
    off = np.frombuffer(b, dtype=np.uint8, count=p * stride, offset=o).reshape(p, stride)[:, :nv]
    o += p * stride
    assert o == len(b)
    return dict(gens=gens, star=star, S=S, f=f, uid=uid, hist=hist, hc=hc, off=off)


def _run_and_checkpoint(g, p, G, depth, seed):
    s = P.Solver(g, depth=depth)
    s.begin(p, seed)
    s.step(G)
    img = s.checkpoint()
    grid, filled = s.end()
    return s, img, grid, filled


def _compare_state(ck, r, hlen=HIST):
    np.testing.assert_array_equal(ck["S"], r["final_S"])
    np.testing.assert_array_equal(ck["f"], r["final_f"])
    np.testing.assert_array_equal(ck["uid"], r["uid"])
    np.testing.assert_array_equal(ck["hc"], r["hcount"])
    # every written history slot (the rest is never read)
    for i in range(len(ck["hc"])):
        k = min(int(ck["hc"][i]), hlen)
        np.testing.assert_array_equal(ck["hist"][i, :k], r["hist"][i, :k])
    np.testing.assert_array_equal(ck["off"], r["offspring"])
    np.testing.assert_array_equal(ck["star"], r["best"])


def test_whole_run_n50_population_256(torch_cuda, oracle_mod):
    """Planted n = 50, 50 % prefilled (the benchmark's grid), p = 256, three
    generations of depth 25000: result, statistics and the state of Alg. 2
    after the run equal the oracle's."""
    w = gen.workload_n50()
    p, G = 256, 3
    _say(f"whole run n50 p={p} G={G} depth={w['depth']}")
    s, img, grid, filled = _run_and_checkpoint(w["grid"], p, G, w["depth"], w["seed"])
    st = s.stats()
    I = oracle_mod.Instance(w["grid"])
    r = I.run_state(I.params(depth=w["depth"]), p, G, w["seed"])
    assert filled == r["filled"]
    np.testing.assert_array_equal(grid, r["grid"])
    np.testing.assert_array_equal(st["best_f_per_gen"], r["best_f"])
    np.testing.assert_array_equal(st["counters_per_gen"], r["counters"])
    ck = parse_checkpoint(img, I.nv)
    assert ck["gens"] == G
    _compare_state(ck, r)


@pytest.mark.parametrize("kind,n,prefill,G", [("greedy", 16, 0.6, 3), ("planted", 12, 0.5, 2)])
def test_whole_run_population_16384(torch_cuda, oracle_mod, kind, n, prefill, G):
    """Population 16384 (2p = 32768 candidates: selection keys sorted in
    global memory, many equal individuals and full close lists), full depth
    10 n^2: every generation's best f and counters and the state after the
    run equal the oracle's whole run."""
    g = gen.random_greedy(n, prefill, 6100 + n) if kind == "greedy" else gen.planted(n, prefill,
                                                                                   6200 + n)
    p, depth, seed = 16384, 10 * n * n, gen.solver_seed(6300 + n)
    _say(f"whole run {kind} n={n} p={p} G={G}")
    s, img, grid, filled = _run_and_checkpoint(g, p, G, depth, seed)
    st = s.stats()
    I = oracle_mod.Instance(g)
    r = I.run_state(I.params(depth=depth), p, G, seed)
    assert filled == r["filled"]
    np.testing.assert_array_equal(grid, r["grid"])
    np.testing.assert_array_equal(st["best_f_per_gen"], r["best_f"])
    np.testing.assert_array_equal(st["counters_per_gen"], r["counters"])
    ck = parse_checkpoint(img, I.nv)
    _compare_state(ck, r)


@pytest.mark.parametrize("prefill", [0.3, 0.5, 0.7])
def test_generation1_n70_full_size_sampled(torch_cuda, oracle_mod, prefill):
    """Random-greedy n = 70 at 30 / 50 / 70 % prefilled, population 16384,
    depth 49000: init and generation-1 searches of the whole population on the
    GPU; sampled slots (both ends, tile and wave boundaries) recomputed by the
    oracle: colourings, f and every counter."""
    w = gen.workload_n70(prefill)
    p = w["population"]
    _say(f"n70 r={prefill} p={p} depth={w['depth']} generation 1 sampled")
    s = P.Solver(w["grid"], depth=w["depth"])
    S0, f0 = s.stage_init(p, w["seed"])
    S1, f1, c1 = s.stage_plits(S0, 1, w["seed"])
    torch_cuda.cuda.synchronize()
    I = oracle_mod.Instance(w["grid"])
    slots = [0, 1, 63, 64, 4097, 9000, 12345, p - 1]
    So, fo = I.init_slots(w["seed"], slots)
    S0h = S0.cpu().numpy()
    np.testing.assert_array_equal(S0h[slots, :I.nv], So)
    S1o, f1o, c1o = I.plits(I.params(depth=w["depth"]), w["seed"], 1, slots, So)
    np.testing.assert_array_equal(S1.cpu().numpy()[slots, :I.nv], S1o)
    np.testing.assert_array_equal(f1.cpu().numpy()[slots], f1o)
    np.testing.assert_array_equal(c1.cpu().numpy()[slots].astype(np.uint64), c1o)
