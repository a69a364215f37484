"""Benchmark: tabu moves/s of the MPMA hot path on one MI355X.

A step is one generation of Alg. 2 over the whole population: PLITS on every
offspring, best-solution saving, Hamming distances over both populations,
population update, parent matching and AUX crossover.  Inputs are resident in
HBM before the timed region; W warmup generations run first, then exactly K
generations are timed (device synchronised on both sides).

value = tabu moves executed in the K timed generations / their wall time.
roofline: the tabu-search kernel's algorithmic state bytes per launch (from
the per-generation counters, see plits_state_bytes; the state is LDS-resident)
over its mean launch time from HIP events recorded on the launch stream.
cpu_baseline: the CPU oracle's PLITS on a bounded sample of the same
generation-1 population, on the host's cores.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# LDS: 256 CUs x 128 B/clk x 2.4 GHz (nominal; the level that holds the state)
LDS_PEAK_GBS = 256 * 128 * 2.4


def plits_state_bytes(cnt, p, n, nv):
    """Algorithmic bytes of search state one tabu-search launch touches.

    The state of an individual is its colouring S (1 B per vertex), the row and
    column colour counts (1 B each), the eligibility bitmap and the tabu table.
    Per iteration: the bitmap (|V|/8 B); per eligible vertex its colour and
    the two counts of that colour (3 B); per candidate move the two counts of
    the candidate colour (2 B).  Per move: four counts read and written (8 B),
    the colour (1 B), one tabu entry (4 B) and the colours of the 2(n-1) row
    and column vertices (2(n-1) B).  Per snapshot |V| B; per phase of every
    individual the start row (|V| B).
    cnt: counters [iters, moves, idle, cands, elig, nupd, snaps, repairs].
    """
    iters, moves, cands, elig, snaps = (int(cnt[0]), int(cnt[1]), int(cnt[3]), int(cnt[4]),
                                        int(cnt[6]))
    return (iters * ((nv + 7) // 8) + elig * 3 + cands * 2 + moves * (13 + 2 * (n - 1))
            + snaps * nv + p * 2 * nv)


def cpu_baseline(grid, seed, depth, target_s=12.0):
    """Oracle PLITS of generation 1 on a bounded sample of slots."""
    from oracle import oracle as O
    O.build()
    I = O.Instance(grid)
    P = I.params(depth=depth)
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    moves = 0
    elapsed = 0.0
    done = 0
    k = threads
    while True:
        slots = list(range(done, done + k))
        S, _ = I.init_slots(seed, slots)
        t0 = time.perf_counter()
        _, _, cnt = I.plits(P, seed, 1, slots, S)
        elapsed += time.perf_counter() - t0
        moves += int(cnt[:, 1].sum())
        done += k
        if elapsed >= target_s * 0.6:
            break
        k = threads * max(1, int(math.ceil((target_s - elapsed) / max(elapsed, 1e-3) * done / threads)))
        k = min(k, 16 * threads)
    return {"value": moves / elapsed, "unit": "moves/s", "cores": threads, "kind": "oracle",
            "sample": f"generation-1 PLITS of slots 0..{done - 1} of the same population "
                      f"({done} individuals, {moves} moves, {elapsed:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n50", choices=["n50", "n70_30", "n70_50", "n70_70",
                                                         "small"])
    ap.add_argument("--lanes-per-vertex", type=int, default=0)
    ap.add_argument("--population", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise device copy of MIB MiB (reads MIB, "
                         "writes MIB), the reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.copy_reference:
        import torch
        n = args.copy_reference * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.add(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes_read": n * 4, "copy_reference_bytes_written": n * 4}))
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not part of it "
              "(see DESIGN.md for how the population would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2103_10453_amd import instances as gen
    from paper_2103_10453_amd import plse

    if args.workload == "n50":
        w = gen.workload_n50()
        desc = "planted n=50, 50% prefilled, population 16384, depth 10n^2 per generation"
    elif args.workload == "small":
        w = gen.workload_small()
        desc = "planted n=10, 40% prefilled, population 64, depth 10n^2 per generation"
    else:
        r = int(args.workload.split("_")[1]) / 100.0
        w = gen.workload_n70(r)
        desc = f"random-greedy n=70, {int(r * 100)}% prefilled, population 16384, depth 10n^2"
    if args.population:
        w["population"] = args.population
    p = w["population"]
    torch.cuda.set_device(0)
    s = plse.Solver(w["grid"], depth=w["depth"], lanes_per_vertex=args.lanes_per_vertex)
    s.ensure_workspace(p)
    stream = torch.cuda.current_stream()

    s.begin(p, w["seed"], stream)
    s.step(args.warmup, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grid, filled = s.end(stream)
    st = s.stats()
    ms_plits, ms_rest = s.timing()
    gens = st["generations_run"]
    cnt = st["counters_per_gen"]
    timed = slice(args.warmup, min(args.warmup + args.steps, gens))
    moves_timed = int(cnt[timed, 1].sum())
    wall = t1 - t0
    value = moves_timed / wall
    bytes_gen = [plits_state_bytes(cnt[g], p, s.n, s.nv) for g in range(timed.start, timed.stop)]
    t_plits = [float(ms_plits[g]) for g in range(timed.start, timed.stop)]
    achieved = (sum(bytes_gen) / max(len(bytes_gen), 1)) / (np.mean(t_plits) * 1e-3) / 1e9
    out = {
        "metric": "tabu moves/s (n=50, pop 16384)" if args.workload == "n50"
        else f"tabu moves/s ({args.workload}, pop {p})",
        "value": value,
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": int(w["grid"].shape[0]), "population": p,
                   "depth": int(w["depth"]),
                   "lanes_per_vertex": int(s.get_param("lanes_per_vertex")),
                   "vertices": s.nv, "sum_domain": s.nd,
                   "waves_per_block": int(s.get_param("waves_per_block"))},
        "roofline": {"bound": "lds", "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / LDS_PEAK_GBS, "traffic": None},
        "detail": {"moves_timed": moves_timed, "plits_ms_per_gen": t_plits,
                   "rest_ms_per_gen": [float(ms_rest[g]) for g in range(timed.start, timed.stop)],
                   "plits_bytes_per_gen": bytes_gen,
                   "moves_per_gen": [int(x) for x in cnt[:, 1]],
                   "iters_per_gen": [int(x) for x in cnt[:, 0]],
                   "best_f_per_gen": [int(x) for x in st["best_f_per_gen"]],
                   "filled": filled, "upper_bound": s.ub,
                   "plits_moves_per_s": moves_timed / (sum(t_plits) * 1e-3)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w["grid"], w["seed"], w["depth"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
