"""Benchmark: tabu moves/s of the MPMA hot path on one MI355X.

A step is one generation of Alg. 2 over the whole population: PLITS on every
offspring, best-solution saving, Hamming distances over both populations,
population update, parent matching and AUX crossover.  Inputs are resident in
HBM before the timed region; W warmup generations run first, then exactly K
generations are timed (device synchronised on both sides).

value = tabu moves executed in the K timed generations / their wall time.
roofline: the tabu-search kernel against the LDS level, where the search
state it touches per move lives: algorithmic bytes per launch from the
per-generation counters (per move: every candidate's conflict and tabu
entries, the conflict-table entries of the moved vertex's neighbours, the
eligibility scan, the colour and tabu writes, snapshots; 2-byte conflict and
tabu entries) over the launch's mean time from HIP events on its stream,
against the LDS read bandwidth measured on this GPU in the same run.  The
same launch's integer-operation rate against the int32 VALU peak is given
beside it.
traffic: HBM bytes per launch from the committed rocprofv3 FETCH_SIZE /
WRITE_SIZE summary of this command, scaled by the copy-kernel factors stated
in it; null when the kernel sources changed since it was taken.
cpu_baseline: the CPU oracle's PLITS on a bounded sample of the offspring the
GPU searched in the first timed generation (read from a checkpoint taken
after the warmup), on the host's cores; the generation-1 pair beside it.
sustained: a few generations of the 70x70 grid 70 % prefilled (p = 16384,
depth 49000), whose searches never complete, so every generation is full.
stages_ms: per-stage GPU times of a separate stage-timed run (plse_last_stage_timing).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import hashlib

HBM_PEAK_GBS = 8000.0
# int32 VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one operation per lane
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PLITS_SOURCES = ["k_plits.hip", "device_common.h", "kernels.h", "plse_internal.h"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "plits_n50_hbm.txt")
# bytes per conflict-table entry and per tabu entry in the algorithmic count
B_CONF, B_TABU = 2, 2


def plits_alg_ops(cnt, n, nv):
    """Algorithmic integer operations of one tabu-search launch.

    Per candidate move (counter cands): 10 -- the move's conflict count from
    the row and column counts (1), its value (1), tabu and aspiration tests
    (3), tie value (1), key (2), keep-the-best comparison and select (2).
    Per eligible vertex (elig): 10 -- its current conflicts (2), its tie hash
    (7), bookkeeping (1).  Per iteration (iters): the eligibility bitmap scan
    (2 per 32 vertices), the colour tie hashes (7 per colour), tenure and
    bookkeeping (10).  Per move (moves): 8 for the counts, colour and
    objective, 3 per row/column vertex re-checked (2|V|/n on average).  Per
    snapshot (snaps): |V|/4 word copies.
    cnt: counters [iters, moves, idle, cands, elig, nupd, snaps, repairs, cupd].
    """
    iters, moves, cands, elig, snaps = (int(cnt[0]), int(cnt[1]), int(cnt[3]), int(cnt[4]),
                                        int(cnt[6]))
    per_iter = 2 * ((nv + 31) // 32) + 7 * (n + 1) + 10
    per_move = 8 + 3 * (2 * nv // n)
    return cands * 10 + elig * 10 + iters * per_iter + moves * per_move + snaps * (nv // 4)


def plits_alg_bytes(cnt, nv):
    """Algorithmic bytes of one tabu-search launch (Section 3.3's incremental
    evaluation): per candidate move its conflict entry and tabu entry read;
    per neighbour of the moved vertex and coloured end of the move, one
    conflict entry read and written; per iteration the eligibility scan
    (|V| / 8); per move the colour and the tabu entry written; per snapshot
    |V| colours.
    cnt: counters [iters, moves, idle, cands, elig, nupd, snaps, repairs, cupd]."""
    iters, moves, cands, nupd, snaps = (int(cnt[0]), int(cnt[1]), int(cnt[3]), int(cnt[5]),
                                        int(cnt[6]))
    return (cands * (B_CONF + B_TABU) + nupd * 2 * B_CONF + iters * ((nv + 7) // 8)
            + moves * (1 + B_TABU) + snaps * nv)


def plits_sources_sha256():
    h = hashlib.sha256()
    for name in PLITS_SOURCES:
        with open(os.path.join(ROOT, "paper_2103_10453_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def plits_traffic(warmup, steps, workload):
    """HBM bytes per timed launch from the committed counter summary, or None."""
    if workload != "n50" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    meta, rows = {}, []
    with open(TRAFFIC_PROFILE) as f:
        for line in f:
            t = line.split()
            if len(t) >= 3 and t[0] == "#" and t[1].endswith(":"):
                meta[t[1][:-1]] = t[2]
            elif len(t) == 4 and t[0].isdigit():
                rows.append((int(t[0]), float(t[2]), float(t[3])))
    if meta.get("kernel_sources_sha256") != plits_sources_sha256():
        return None
    if int(meta.get("warmup", -1)) != warmup or int(meta.get("steps", -1)) != steps:
        return None
    ff, wf = float(meta["fetch_factor"]), float(meta["write_factor"])
    timed = [r for r in rows if warmup < r[0] <= warmup + steps]
    if len(timed) != steps:
        return None
    return sum((fk * ff + wk * wf) * 1024.0 for _, fk, wk in timed) / steps


def host_cpu():
    """Model name and logical CPUs of the host (lscpu)."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:
        return None
    info = {}
    for line in out.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Socket(s)"):
                info[k.strip()] = v.strip()
    return info


def _oracle_rate(I, P, seed, gen_no, S_rows, threads, target_s, label):
    """Oracle PLITS moves/s over leading rows of S_rows, sized to ~target_s."""
    moves, elapsed, done = 0, 0.0, 0
    k = threads
    while done < len(S_rows):
        k = min(k, len(S_rows) - done)
        slots = list(range(done, done + k))
        t0 = time.perf_counter()
        _, _, cnt = I.plits(P, seed, gen_no, slots, S_rows[done:done + k])
        elapsed += time.perf_counter() - t0
        moves += int(cnt[:, 1].sum())
        done += k
        if elapsed >= target_s * 0.6:
            break
        k = threads * max(1, int(math.ceil((target_s - elapsed) / max(elapsed, 1e-3) * done / threads)))
        k = min(k, 16 * threads)
    return {"value": moves / elapsed, "sample": f"{label}: slots 0..{done - 1} ({done} individuals, "
                                                f"{moves} moves, {elapsed:.1f} s)"}


def cpu_baseline(grid, seed, depth, gen_no, offspring, gpu_gen1, target_s=10.0):
    """The oracle's PLITS on the offspring of generation gen_no (the first
    timed generation), and on the initial population (generation 1)."""
    from oracle import oracle as O
    O.build()
    I = O.Instance(grid)
    P = I.params(depth=depth)
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    r = _oracle_rate(I, P, seed, gen_no, offspring, threads, target_s,
                     f"generation-{gen_no} PLITS of the GPU's offspring")
    S1, _ = I.init_slots(seed, list(range(min(4096, len(offspring)))))
    r1 = _oracle_rate(I, P, seed, 1, S1, threads, target_s, "generation-1 PLITS")
    return {"value": r["value"], "unit": "moves/s", "cores": threads, "kind": "oracle",
            "sample": r["sample"], "host": host_cpu(),
            "generation1": {"oracle_moves_per_s": r1["value"], "sample": r1["sample"],
                            "gpu_moves_per_s": gpu_gen1}}


def sustained_run(gen, plse, warmup=1, steps=3):
    """Generations of the 70x70 grid 70 % prefilled, whose searches all run
    to their full depth: moves/s with every generation busy."""
    import torch
    w = gen.workload_n70(0.7)
    p = w["population"]
    s = plse.Solver(w["grid"], depth=w["depth"])
    s.ensure_workspace(p)
    stream = torch.cuda.current_stream()
    s.begin(p, w["seed"], stream)
    s.step(warmup, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.end(stream)
    st = s.stats()
    ms_plits, _ = s.timing()
    cnt = st["counters_per_gen"][warmup:warmup + steps]
    moves = int(cnt[:, 1].sum())
    out = {"workload": "random-greedy n=70, 70% prefilled, population 16384, depth 49000",
           "warmup": warmup, "steps": steps, "moves_per_s": moves / wall,
           "ms_per_step": wall / steps * 1e3,
           "plits_ms_per_gen": [float(x) for x in ms_plits[warmup:warmup + steps]],
           "moves_per_gen": [int(x) for x in cnt[:, 1]],
           "best_f_per_gen": [int(x) for x in st["best_f_per_gen"]]}
    del s
    torch.cuda.empty_cache()
    return out


def stage_times(plse, w, p, G=3):
    """Per-stage GPU times of a stage-timed run of the same workload."""
    s = plse.Solver(w["grid"], depth=w["depth"], stage_timing=1)
    s.solve(p, G, w["seed"])
    st = s.stage_timing()
    return {"generations": G, "mean_ms_after_generation_1": {
        name: float(st[1:, i].mean()) for i, name in enumerate(plse.STAGES)},
        "generation_1_ms": {name: float(st[0, i]) for i, name in enumerate(plse.STAGES)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n50", choices=["n50", "n70_30", "n70_50", "n70_70",
                                                         "n70_80", "small", "batch", "served",
                                                         "lsc"])
    ap.add_argument("--variant", type=int, default=0, choices=[0, 1],
                    help="0 MPMA, 1 Partial-MPMA (repair + PartialCol)")
    ap.add_argument("--instances", type=int, default=256, help="batch: number of instances")
    ap.add_argument("--autotune", action="store_true",
                    help="batch: pick each instance's launch shape by measurement first")
    ap.add_argument("--batch-part", default="both", choices=["both", "batched", "sequential"],
                    help="batch: run both halves, or one (see --results-file)")
    ap.add_argument("--batch-chunk", type=int, default=5,
                    help="batch: generations stepped between progress lines")
    ap.add_argument("--results-file", default="",
                    help="batch with one half: save its grids here, or compare with the "
                         "other half's saved grids if the file exists; served: where the "
                         "solo part saves its results and the served part reads them")
    ap.add_argument("--requests", type=int, default=64, help="served: number of requests")
    ap.add_argument("--rate", type=float, default=20.0, help="served: arrivals per second")
    ap.add_argument("--rates", default="",
                    help="served: comma-separated arrival rates (one JSON line each)")
    ap.add_argument("--served-part", default="both", choices=["both", "solo", "served"],
                    help="served: run the solo baseline, the served streams, or both "
                         "(see --results-file)")
    ap.add_argument("--max-slots", type=int, default=0,
                    help="served: requests resident at once (admission limit; 0: one per "
                         "hardware queue, since requests sharing a queue wait for each other)")
    ap.add_argument("--generations", type=int, default=0,
                    help="served: generations per request (default 50)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="served: hardware queues of the process (GPU_MAX_HW_QUEUES, at most "
                         "32), so that resident requests' streams run side by side (HIP's "
                         "default is 4); 0 keeps the environment's value")
    ap.add_argument("--slots-per-lane", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--population", type=int, default=0)
    ap.add_argument("--plits-kernel", type=int, default=0, choices=[0, 1, 2],
                    help="tabu-search kernel: 0/1 global tabu table, 2 LDS-resident")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sustained", action="store_true",
                    help="skip the sustained-throughput generations of the 70x70 grid")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise device copy of MIB MiB (reads MIB, "
                         "writes MIB), the reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.workload == "served" and args.hw_queues > 0:
        # read by the HIP runtime when it initialises, which is later (torch
        # is imported lazily); --hw-queues 0 keeps the environment's value
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.hw_queues, 32))
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
        print("bench.py: runs on one GPU only; across GPUs the population would shard by "
              "individual with one all-gather of the offspring per generation", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2103_10453_amd import instances as gen
    from paper_2103_10453_amd import plse

    if args.workload == "batch":
        return bench_batch(args, gen, plse)
    if args.workload == "served":
        return bench_served(args, gen, plse)
    if args.workload == "lsc":
        return bench_lsc(args, gen, plse)
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
    if args.variant:
        desc += ", Partial-MPMA"
    if args.population:
        w["population"] = args.population
    p = w["population"]
    torch.cuda.set_device(0)
    s = plse.Solver(w["grid"], depth=w["depth"], slots_per_lane=args.slots_per_lane,
                    waves_per_block=args.waves_per_block, variant=args.variant,
                    plits_kernel=args.plits_kernel)
    s.ensure_workspace(p)
    stream = torch.cuda.current_stream()

    s.begin(p, w["seed"], stream)
    s.step(args.warmup, stream)
    torch.cuda.synchronize()
    # the offspring the first timed generation searches (for the CPU
    # baseline); the image ends with them (include/plse.h)
    offspring = None
    if not args.no_cpu_baseline and args.workload == "n50" and args.warmup >= 1:
        img = s.checkpoint(stream)
        offspring = np.asarray(img[len(img) - p * s.stride:]).reshape(p, s.stride)[:, :s.nv].copy()
        del img
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
    t_plits = [float(ms_plits[g]) for g in range(timed.start, timed.stop)]
    t_mean = np.mean(t_plits) * 1e-3
    bytes_gen = [plits_alg_bytes(cnt[g], s.nv) for g in range(timed.start, timed.stop)]
    ops_gen = [plits_alg_ops(cnt[g], s.n, s.nv) for g in range(timed.start, timed.stop)]
    b_launch = sum(bytes_gen) / max(len(bytes_gen), 1)
    achieved = b_launch / t_mean / 1e9
    alu = (sum(ops_gen) / max(len(ops_gen), 1)) / t_mean / 1e12
    lds_peak = plse.plse_measure_lds_bandwidth(5) / 1e9
    traffic = plits_traffic(args.warmup, args.steps, args.workload)
    kernel = "plits_%skernel<%d%s>" % ("lean_" if s.get_param("plits_kernel") == 2 else "",
                                       int(s.get_param("slots_per_lane")),
                                       "" if s.get_param("plits_kernel") == 2 else
                                       (", true" if args.variant else ", false"))
    out = {
        "metric": "tabu moves/s (n=50, pop 16384)" if args.workload == "n50" and not args.variant
        else f"tabu moves/s ({args.workload}{', Partial-MPMA' if args.variant else ''}, pop {p})",
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
                   "slots_per_lane": int(s.get_param("slots_per_lane")),
                   "vertices": s.nv, "sum_domain": s.nd,
                   "waves_per_block": int(s.get_param("waves_per_block")),
                   "resident_waves_per_cu": int(s.get_param("plits_waves_per_cu"))},
        "roofline": {"bound": "lds", "achieved": achieved, "peak": lds_peak, "unit": "GB/s",
                     "frac": achieved / lds_peak, "traffic": traffic, "kernel": kernel,
                     "bytes_per_launch": b_launch,
                     "bytes_per_move": b_launch / max(moves_timed / max(len(bytes_gen), 1), 1),
                     "launch_ms": t_mean * 1e3,
                     "peak_source": "plse_measure_lds_bandwidth: conflict-free 16-byte LDS "
                                    "reads on every CU, this GPU, this run",
                     "hbm_gbs": (traffic / t_mean / 1e9) if traffic else None,
                     "hbm_frac": (traffic / t_mean / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "alu": {"achieved": alu, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                             "frac": alu / ALU_PEAK_TOPS}},
        "detail": {"moves_timed": moves_timed, "plits_ms_per_gen": t_plits,
                   "rest_ms_per_gen": [float(ms_rest[g]) for g in range(timed.start, timed.stop)],
                   "plits_alg_bytes_per_gen": bytes_gen,
                   "plits_alg_ops_per_gen": ops_gen,
                   "moves_per_gen": [int(x) for x in cnt[:, 1]],
                   "iters_per_gen": [int(x) for x in cnt[:, 0]],
                   "cands_per_gen": [int(x) for x in cnt[:, 3]],
                   "elig_per_gen": [int(x) for x in cnt[:, 4]],
                   "nupd_per_gen": [int(x) for x in cnt[:, 5]],
                   "snaps_per_gen": [int(x) for x in cnt[:, 6]],
                   "best_f_per_gen": [int(x) for x in st["best_f_per_gen"]],
                   "filled": filled, "upper_bound": s.ub,
                   "plits_moves_per_s": moves_timed / (sum(t_plits) * 1e-3),
                   # generation 1 (the first warm-up step): every search busy
                   "first_generation": ({"moves": int(cnt[0, 1]), "plits_ms": float(ms_plits[0]),
                                         "moves_per_s": float(cnt[0, 1]) / (float(ms_plits[0]) * 1e-3)}
                                        if args.warmup >= 1 and gens >= 1 else None)},
    }
    del s
    torch.cuda.empty_cache()
    if args.workload == "n50" and not args.variant:
        out["stages_ms"] = stage_times(plse, w, p)
        if not args.no_sustained:
            out["sustained"] = sustained_run(gen, plse)
    if offspring is not None:
        g1 = out["detail"]["first_generation"]
        out["cpu_baseline"] = cpu_baseline(w["grid"], w["seed"], w["depth"], args.warmup + 1,
                                           offspring, g1["moves_per_s"] if g1 else None)
    print(json.dumps(out), flush=True)


def bench_batch(args, gen, plse):
    """Many instances at once (batched session: per generation one persistent
    search launch per launch-shape group) vs one plse_solve per instance, same
    seeds and generations: results must be identical.  Both halves report
    progress as they go; --batch-part runs one half (results saved to / compared
    with --results-file) so that long configurations fit separate runs."""
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    work = gen.workload_batch(args.instances)
    G = args.steps
    solvers = [plse.Solver(w["grid"], depth=w["depth"]) for w in work]
    p = work[0]["population"]
    seeds = [w["seed"] for w in work]
    ns = [int(w["grid"].shape[0]) for w in work]
    for s in solvers:
        s.ensure_workspace(p)
    t_tune = None
    if args.autotune:
        # measured launch shapes per instance (results do not depend on them)
        t0 = time.perf_counter()
        for s, w in zip(solvers, work):
            s.autotune_shape(sample=p, depth=500, seed=w["seed"])
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
    shapes = {}
    for s in solvers:
        k = f"{s.get_param('slots_per_lane')}x{s.get_param('waves_per_block')}"
        shapes[k] = shapes.get(k, 0) + 1
    out = {"metric": f"batched tabu moves/s ({len(work)} instances, pop {p}, {G} generations)",
           "value": None, "unit": "moves/s", "n_gpus": 1, "steps": G, "warmup": 0,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "batch: n ~ U{20..70}, r ~ U[0.3, 0.7], half planted, half "
                                  "random-greedy, population 1024, depth 10n^2",
                      "instances": len(work), "population": p,
                      "launch_shapes": "autotuned" if args.autotune else "cost model",
                      "search_launch": "one persistent launch per launch-shape group and "
                                       "generation, waves taking (instance, individual) items "
                                       "longest estimated work first"},
           "shapes": shapes, "autotune_seconds": t_tune}
    res_b = res_s = None
    stream = torch.cuda.current_stream()
    if args.batch_part in ("both", "batched"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = plse.plse_batch_begin([s.h for s in solvers], p, seeds, stream)
        done = 0
        while done < G:
            k = min(args.batch_chunk, G - done)
            plse.plse_batch_step(b, k, stream)
            torch.cuda.synchronize()
            done += k
            print(f"[batch] batched: {done}/{G} generations, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
        res_b = plse.plse_batch_end(b, ns, stream)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        moves_b = sum(int(s.stats()["totals"][1]) for s in solvers)
        out.update({"value": moves_b / t_batch, "ms_per_step": t_batch / G * 1e3,
                    "batched_seconds": t_batch, "batched_moves": moves_b})
    if args.batch_part in ("both", "sequential"):
        t0 = time.perf_counter()
        res_s = []
        for i, (s, w) in enumerate(zip(solvers, work)):
            res_s.append(s.solve(p, G, w["seed"]))
            if (i + 1) % 16 == 0 or i + 1 == len(work):
                print(f"[batch] one instance per launch: {i + 1}/{len(work)} instances, "
                      f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        moves_s = sum(int(s.stats()["totals"][1]) for s in solvers)
        out["one_instance_per_launch"] = {"value": moves_s / t_seq, "seconds": t_seq,
                                          "moves": moves_s}
    mine = res_b if res_b is not None else res_s
    if args.results_file and args.batch_part != "both":
        other = args.results_file if os.path.exists(args.results_file) else None
        if other is None:
            np.savez(args.results_file, filled=np.array([r[1] for r in mine]),
                     **{f"g{i}": r[0] for i, r in enumerate(mine)})
        else:
            z = np.load(other)
            out["identical_results"] = bool(all(
                int(z["filled"][i]) == r[1] and np.array_equal(z[f"g{i}"], r[0])
                for i, r in enumerate(mine)))
            out["compared_with"] = os.path.basename(other)
    if res_b is not None and res_s is not None:
        out["speedup"] = out["one_instance_per_launch"]["seconds"] / out["batched_seconds"]
        out["identical_results"] = all(a[1] == b_[1] and np.array_equal(a[0], b_[0])
                                       for a, b_ in zip(res_b, res_s))
    out["filled_total"] = int(sum(r[1] for r in mine))
    print(json.dumps(out), flush=True)


def bench_lsc(args, gen, plse):
    """Latin square completion mode: planted instances (completable by
    construction) solved with the stop at the bound, i.e. at f = 0; reports
    success, generations and time to a complete square."""
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    p = args.population or 4096
    G = args.generations or 50
    cases = [(50, 0.5), (60, 0.5), (70, 0.5), (60, 0.4)]
    rows, moves, t_all = [], 0, 0.0
    for k, (n, r) in enumerate(cases):
        g = gen.planted(n, r, 7000 + k)
        s = plse.Solver(g, depth=10 * n * n, stop_at_ub=1)
        s.solve(p, 1, 1)  # warm-up: workspace and code
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        grid, filled = s.solve(p, G, 9000 + k)
        t = time.perf_counter() - t0
        st = s.stats()
        ok = filled == n * n and gen.is_partial_latin(grid)
        moves += int(st["totals"][1])
        t_all += t
        rows.append({"n": n, "prefill": r, "solved": bool(ok),
                     "generations": int(st["generations_run"]), "seconds": t})
    print(json.dumps({
        "metric": f"LSC: planted instances completed (pop {p}, at most {G} generations)",
        "value": sum(r["solved"] for r in rows) / len(rows), "unit": "fraction solved",
        "n_gpus": 1, "steps": G, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "lsc: planted (n, prefill) in " + str(cases)
                               + ", depth 10n^2, stop at f = 0", "population": p},
        "moves_per_s": moves / t_all if t_all else None, "cases": rows}), flush=True)


def fifo_latencies(arrival, service):
    """One request at a time in arrival order: start = max(arrival, previous
    finish), finish = start + service; returns (start, finish)."""
    start, finish, t = [], [], 0.0
    for a, sv in zip(arrival, service):
        st = max(a, t)
        t = st + sv
        start.append(st)
        finish.append(t)
    return start, finish


def bench_served(args, gen, plse):
    """Poisson request streams through the continuous-batching server vs the
    same streams served one request at a time; same results required.

    The request set is the same at every rate (the gaps rescale).  Serving
    one request at a time is measured once: each request solved alone on the
    otherwise idle GPU (its solver and workspace prepared before its timer),
    giving its service time and the offset of its best generation; the
    one-at-a-time latencies of each rate follow by replaying the arrivals
    through a single first-come first-served server with those service times.
    --served-part solo / served splits the two halves over runs (the solo
    results go to --results-file)."""
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    G = args.generations or 50
    rates = [float(x) for x in args.rates.split(",")] if args.rates else [args.rate]
    unit = gen.workload_served(args.requests, 1.0)
    p = unit[0]["population"]
    pct = lambda a, q: float(np.percentile(a, q))
    solvers = [plse.Solver(r["grid"], depth=r["depth"], max_generations=G) for r in unit]
    solo = None
    if args.served_part in ("both", "solo"):
        svc, ttb_off, grids, filled, moves = [], [], [], [], 0
        t_all = time.perf_counter()
        for k, (s, r) in enumerate(zip(solvers, unit)):
            s.ensure_workspace(p)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g, f = s.solve(p, G, r["seed"])
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = s.stats()
            ms_p, ms_r = s.timing()
            per_gen = (np.asarray(ms_p) + np.asarray(ms_r)) * 1e-3
            setup = max(wall - float(per_gen.sum()), 0.0)
            bg = max(int(st["best_generation"]), 1)
            svc.append(wall)
            ttb_off.append(setup + float(per_gen[:bg].sum()))
            grids.append(g)
            filled.append(f)
            moves += int(st["totals"][1])
            # the workspace goes before the next request's (and the server's arena)
            plse.plse_attach_workspace(s.h, None)
            s._ws = None
            torch.cuda.empty_cache()
            print(f"[served] solo {k + 1}/{len(unit)}: n={r['grid'].shape[0]} {wall:.2f} s "
                  f"(total {time.perf_counter() - t_all:.1f} s)", file=sys.stderr, flush=True)
        solo = dict(service=np.array(svc), ttb=np.array(ttb_off),
                    filled=np.array(filled), moves=moves, grids=grids)
        if args.results_file:
            np.savez(args.results_file, service=solo["service"], ttb=solo["ttb"],
                     filled=solo["filled"], moves=np.array([moves]),
                     **{f"g{i}": g for i, g in enumerate(grids)})
    elif args.results_file and os.path.exists(args.results_file):
        z = np.load(args.results_file)
        solo = dict(service=z["service"], ttb=z["ttb"], filled=z["filled"],
                    moves=int(z["moves"][0]), grids=[z[f"g{i}"] for i in range(len(unit))])
    if args.served_part == "solo":
        print(json.dumps({"metric": f"solo service times ({len(unit)} requests, pop {p}, "
                                    f"{G} generations)", "value": float(solo["service"].sum()),
                          "unit": "s", "mean_s": float(solo["service"].mean()),
                          "moves_per_s": solo["moves"] / float(solo["service"].sum())}),
              flush=True)
        return
    free = torch.cuda.mem_get_info()[0]
    budget = int(0.7 * free) // 256 * 256
    max_slots = args.max_slots or int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    for rate in rates:
        reqs = [dict(r, arrival=r["arrival"] / rate) for r in unit]
        srv = plse.Server(budget, max_slots=max_slots)
        tickets, results = [], {}
        t0 = time.perf_counter()
        i = 0
        while len(results) < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i]["arrival"] <= now:
                tickets.append((i, srv.submit(solvers[i], p, G, reqs[i]["seed"])))
                i += 1
            for k, t in tickets:
                if k not in results:
                    r = srv.poll(t)
                    if r is not None:
                        results[k] = r
                        print(f"[served] rate {rate:g}: {len(results)}/{len(reqs)} done, "
                              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
            time.sleep(0.001)
        wall = time.perf_counter() - t0
        srv.close()
        del srv
        torch.cuda.empty_cache()
        lat = np.array([results[k]["done_s"] - results[k]["submit_s"] for k in range(len(reqs))])
        ttb = np.array([results[k]["best_s"] - results[k]["submit_s"] for k in range(len(reqs))])
        moves = sum(results[k]["moves"] for k in range(len(reqs)))
        row = {
            "metric": f"served requests/s (Poisson {rate:g}/s, {len(reqs)} requests, pop {p}, "
                      f"{G} generations)",
            "value": len(reqs) / wall, "unit": "requests/s", "n_gpus": 1, "steps": G,
            "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": "served: n ~ U{10..100}, r ~ U[0.3, 0.7], planted or "
                                   "random-greedy, population 2048, depth 10n^2",
                       "requests": len(reqs), "rate": rate, "generations": G,
                       "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                       "max_slots": max_slots, "arena_bytes": budget},
            "wall_s": wall, "moves_per_s": moves / wall,
            "latency_s": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
            "time_to_best_s": {"p50": pct(ttb, 50), "p99": pct(ttb, 99)}}
        if solo is not None:
            arr = [r["arrival"] for r in reqs]
            st, fin = fifo_latencies(arr, solo["service"])
            lat_b = np.array(fin) - np.array(arr)
            ttb_b = np.array(st) + solo["ttb"] - np.array(arr)
            row["one_at_a_time"] = {
                "requests_per_s": len(reqs) / (fin[-1] - arr[0] if len(arr) else 1.0),
                "moves_per_s": solo["moves"] / float(solo["service"].sum()),
                "latency_s": {"p50": pct(lat_b, 50), "p99": pct(lat_b, 99)},
                "time_to_best_s": {"p50": pct(ttb_b, 50), "p99": pct(ttb_b, 99)},
                "method": "solo service times replayed first-come first-served"}
            row["identical_results"] = bool(all(
                results[k]["filled"] == int(solo["filled"][k]) and
                np.array_equal(results[k]["grid"], solo["grids"][k]) for k in range(len(reqs))))
        print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
