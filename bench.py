"""Benchmark: tabu moves/s of the MPMA hot path on one MI355X.

A step is one generation of Alg. 2 over the whole population: PLITS on every
offspring, best-solution saving, Hamming distances over both populations,
population update, parent matching and AUX crossover.  Inputs are resident in
HBM before the timed region; W warmup generations run first, then exactly K
generations are timed (device synchronised on both sides).

value = tabu moves executed in the K timed generations / their wall time.
roofline: the tabu-search kernel's algorithmic HBM bytes per launch (from the
per-generation counters, see plits_hbm_bytes) over its mean launch time from
HIP events recorded on the launch stream.
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


def plits_hbm_bytes(cnt, p, nv, nd, conf_bytes, tabu_bytes=4):
    """Algorithmic HBM bytes of one tabu-search launch (one generation).

    Per iteration each candidate one-move reads its conflict entry and its tabu
    entry; each move read-modify-writes the conflict entries of the moved
    vertex's neighbours and writes one tabu entry; each snapshot writes |V|
    bytes.  Each of the two phases of every individual rebuilds its conflict
    table, clears its tabu table and reads its start row.
    cnt: counters [iters, moves, idle, cands, elig, nupd, snaps, repairs].
    """
    cands, moves, nupd, snaps = int(cnt[3]), int(cnt[1]), int(cnt[5]), int(cnt[6])
    per_move = cands * (conf_bytes + tabu_bytes) + nupd * 2 * conf_bytes + moves * tabu_bytes \
        + snaps * nv
    setup = p * 2 * (nd * conf_bytes + (nd + nv) * tabu_bytes + nv)
    return per_move + setup


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
    ap.add_argument("--conf-bytes", type=int, default=2)
    ap.add_argument("--population", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
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
    s = plse.Solver(w["grid"], depth=w["depth"], conf_bytes=args.conf_bytes)
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
    bytes_gen = [plits_hbm_bytes(cnt[g], p, s.nv, s.nd, args.conf_bytes)
                 for g in range(timed.start, timed.stop)]
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
                   "depth": int(w["depth"]), "conf_bytes": args.conf_bytes,
                   "vertices": s.nv, "sum_domain": s.nd,
                   "waves_per_block": int(s.get_param("waves_per_block"))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
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
