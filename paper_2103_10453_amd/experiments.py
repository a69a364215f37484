"""Paper-style runs and statistics over the GPU solver.

Section 4.3 solves every instance several times (5 runs), each run capped at
a total number of tabu iterations, and reports per instance the best and the
average score over the runs (f_best, f_avg), the mean time and the mean
number of tabu iterations each run needed to reach its own best (Tables 3
and 4, Appendix A), marking scores that reach the upper bound of Section 2.2
as optimal.  Section 5.1 varies the population size under a fixed budget per
run and plots the mean score and the mean iterations to the best.

This module drives those protocols on the library: every generation runs in
the HIP kernels behind the C ABI (plse_begin / plse_step / plse_peek /
plse_end); Python only chooses seeds, stops runs and aggregates.  The
iteration budget is the library's own `max_iterations` parameter (applied at
generation ends, so a run may overshoot it by less than one generation); a
wall-clock budget is applied between generations through plse_peek.

Command line:
  python -m paper_2103_10453_amd.experiments table --n 50 --r 0.7 --instances 3
  python -m paper_2103_10453_amd.experiments sweep --n 60 --r 0.7 \\
      --populations 64,256,1024,4096 --max-iterations 2e9
"""

from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

from . import instances
from . import plse as P

STOP_NONE, STOP_BOUND, STOP_BUDGET, STOP_TIME = 0, 1, 2, 3


@dataclasses.dataclass
class Trial:
    """One run of the memetic algorithm on one instance."""
    seed: int
    filled: int               # score: non-empty cells of the best grid
    upper_bound: int
    generations: int          # generations run
    best_generation: int      # generation whose best is the run's best (0: none)
    iterations: int           # tabu iterations of the whole population
    iterations_to_best: int   # ... up to the end of best_generation
    seconds: float            # wall time of the run (begin .. end)
    seconds_to_best: float    # GPU time of generations 1..best_generation
    stop_reason: int          # STOP_*
    grid: np.ndarray = dataclasses.field(repr=False, default=None)


def trial_record(seed, filled, upper_bound, stats, plits_ms, rest_ms, seconds, stop_reason,
                 grid=None) -> Trial:
    """Build a Trial from the library's per-generation statistics.

    The iterations to the best are the population's iterations summed over
    generations 1..best_generation (the generation at whose end the final S*
    first appeared); the time to the best sums the same generations' GPU
    times (tabu search plus the rest of the generation), without the
    initial population's construction.
    """
    bg = int(stats["best_generation"])
    it = np.asarray(stats["counters_per_gen"], dtype=np.uint64).reshape(-1, P.NCOUNTERS)[:, 0]
    gpu = np.asarray(plits_ms, dtype=np.float64) + np.asarray(rest_ms, dtype=np.float64)
    return Trial(seed=int(seed), filled=int(filled), upper_bound=int(upper_bound),
                 generations=int(stats["generations_run"]), best_generation=bg,
                 iterations=int(it.sum()), iterations_to_best=int(it[:bg].sum()),
                 seconds=float(seconds), seconds_to_best=float(gpu[:bg].sum()) / 1e3,
                 stop_reason=int(stop_reason), grid=grid)


def generation_records(stats, plits_ms, rest_ms, n_cells: int, impossible: int) -> list[dict]:
    """One record per generation of a run: generation, best f, score (filled
    cells of S* = n^2 - l - f), the eight counters and the generation's GPU
    times (tabu search, rest of the generation) in ms.  Timings cover the
    generations stepped in the session; earlier ones (before a resume) get
    None."""
    cnt = np.asarray(stats["counters_per_gen"], dtype=np.uint64).reshape(-1, P.NCOUNTERS)
    names = ["iterations", "moves", "idle", "candidates", "eligible", "updates", "snapshots",
             "repairs"]
    g = int(stats["generations_run"])
    off = g - len(plits_ms)
    out = []
    for k in range(g):
        f = int(stats["best_f_per_gen"][k])
        rec = dict(generation=k + 1, best_f=f, score=n_cells - impossible - f)
        rec.update({nm: int(cnt[k, q]) for q, nm in enumerate(names)})
        t = k - off
        rec["plits_ms"] = float(plits_ms[t]) if 0 <= t < len(plits_ms) else None
        rec["rest_ms"] = float(rest_ms[t]) if 0 <= t < len(rest_ms) else None
        out.append(rec)
    return out


def run_trials(grid, runs: int = 5, population: int = 1024, generations: int = 1000,
               seed: int = 1, max_iterations: int = 0, time_limit_s: float | None = None,
               chunk: int = 1, log=None, gen_log=None, **params) -> list[Trial]:
    """`runs` independent runs on one instance (seeds seed, seed+1, ...).

    Each run stops after `generations`, or at the iteration budget, or, with
    `time_limit_s`, at the first generation boundary past the wall-clock
    limit (checked every `chunk` generations), or at the bound with
    stop_at_ub=1.
    """
    s = P.Solver(np.asarray(grid, dtype=np.int8), max_iterations=int(max_iterations), **params)
    out = []
    for r in range(runs):
        sd = seed + r
        t0 = time.perf_counter()
        s.begin(population, sd)
        reason = STOP_NONE
        if time_limit_s is None:
            s.step(generations)
        else:
            done = 0
            while done < generations:
                k = min(chunk, generations - done)
                s.step(k)
                done += k
                pr = s.peek()
                if pr["stop_reason"]:
                    break
                if time.perf_counter() - t0 >= time_limit_s:
                    reason = STOP_TIME
                    break
        g, filled = s.end()
        secs = time.perf_counter() - t0
        st = s.stats()
        tp, tr = s.timing()
        out.append(trial_record(sd, filled, s.ub, st, tp, tr, secs,
                                st["stop_reason"] or reason, grid=g))
        if log:
            log(f"  run seed {sd}: filled {filled} of bound {s.ub}, {st['generations_run']} "
                f"generations, {secs:.1f} s")
        if gen_log:
            for rec in generation_records(st, tp, tr, s.n * s.n, s.l):
                gen_log(dict(seed=sd, upper_bound=s.ub, **rec))
    return out


def summarize(trials: list[Trial]) -> dict:
    """Per-instance columns of Tables 3-4 and Appendix A: f_best and f_avg over
    the runs, mean time and mean iterations to each run's best, and whether
    f_best reaches the upper bound (an optimal score)."""
    if not trials:
        raise ValueError("no trials")
    f = np.array([t.filled for t in trials], dtype=np.float64)
    ub = trials[0].upper_bound
    return dict(runs=len(trials), upper_bound=ub, f_best=int(f.max()), f_avg=float(f.mean()),
                t_best_s=float(np.mean([t.seconds_to_best for t in trials])),
                nb_iter=float(np.mean([t.iterations_to_best for t in trials])),
                optimal=bool(int(f.max()) == ub),
                generations=float(np.mean([t.generations for t in trials])))


def benchmark_instances(n: int, r: float, count: int, base: int = 5000) -> list[np.ndarray]:
    """Synthetic stand-ins for the (n, r) family of the benchmark of Section
    4.1 (random-greedy construction; instance k has seed base + 100 n + k)."""
    return [instances.random_greedy(n, r, base + 100 * n + k) for k in range(count)]


def table(grids, runs=5, population=1024, generations=1000, seed=1, max_iterations=0,
          time_limit_s=None, log=None, gen_log=None, **params) -> list[dict]:
    """One row per instance: summarize() of `runs` trials.  `log`, if given,
    receives a progress line after each instance."""
    rows = []
    for i, g in enumerate(grids):
        tr = run_trials(g, runs, population, generations, seed + 1000 * i, max_iterations,
                        time_limit_s, log=log,
                        gen_log=(lambda r, i=i: gen_log(dict(instance=i, population=population,
                                                             **r))) if gen_log else None,
                        **params)
        rows.append(dict(instance=i, n=int(np.asarray(g).shape[0]), **summarize(tr)))
        if log:
            log(f"population {population} instance {i}: f_best {rows[-1]['f_best']} "
                f"f_avg {rows[-1]['f_avg']:.2f}")
    return rows


def population_sweep(grids, populations, runs=5, generations=1000, seed=1, max_iterations=0,
                     time_limit_s=None, log=None, **params) -> list[dict]:
    """Section 5.1: for each population size, the mean over instances of f_avg
    and f_best, the mean iterations and time to the best, and how many
    instances reach the best score found by any population size."""
    per_p = {}
    for p in populations:
        per_p[p] = table(grids, runs, p, generations, seed, max_iterations, time_limit_s, log,
                         **params)
    best = [max(per_p[p][i]["f_best"] for p in populations) for i in range(len(grids))]
    rows = []
    for p in populations:
        t = per_p[p]
        rows.append(dict(population=int(p),
                         f_avg=float(np.mean([x["f_avg"] for x in t])),
                         f_best=float(np.mean([x["f_best"] for x in t])),
                         nb_iter=float(np.mean([x["nb_iter"] for x in t])),
                         t_best_s=float(np.mean([x["t_best_s"] for x in t])),
                         reach_best=int(sum(x["f_best"] == b for x, b in zip(t, best)))))
    return rows


def _fmt_table(rows) -> str:
    lines = [f"{'id':>3} {'UB':>6} {'f_best':>7} {'f_avg':>9} {'t(s)':>8} {'nb_iter':>12} {'gens':>6}"]
    for x in rows:
        star = "*" if x["optimal"] else " "
        lines.append(f"{x['instance']:>3} {x['upper_bound']:>6} {x['f_best']:>6}{star} "
                     f"{x['f_avg']:>9.2f} {x['t_best_s']:>8.2f} {x['nb_iter']:>12.4g} "
                     f"{x['generations']:>6.1f}")
    return "\n".join(lines)


def _fmt_sweep(rows) -> str:
    lines = [f"{'p':>6} {'f_avg':>9} {'f_best':>9} {'nb_iter':>12} {'t(s)':>8} {'reach':>5}"]
    for x in rows:
        lines.append(f"{x['population']:>6} {x['f_avg']:>9.2f} {x['f_best']:>9.2f} "
                     f"{x['nb_iter']:>12.4g} {x['t_best_s']:>8.2f} {x['reach_best']:>5}")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("mode", choices=["table", "sweep"])
    ap.add_argument("--n", type=int, default=50)
    ap.add_argument("--r", type=float, default=0.7)
    ap.add_argument("--instances", type=int, default=3)
    ap.add_argument("--runs", type=int, default=5)
    ap.add_argument("--population", type=int, default=1024)
    ap.add_argument("--populations", default="64,256,1024,4096")
    ap.add_argument("--generations", type=int, default=1000, help="generation cap per run")
    ap.add_argument("--max-iterations", type=float, default=0,
                    help="tabu-iteration budget per run (0: none)")
    ap.add_argument("--time-limit", type=float, default=None, help="seconds per run")
    ap.add_argument("--depth", type=int, default=0, help="iterations per individual and "
                    "generation (default 10 n^2)")
    ap.add_argument("--variant", type=int, default=0, help="1: Partial-MPMA")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--json", action="store_true", help="one JSON line per row")
    ap.add_argument("--log", default=None, metavar="FILE",
                    help="table: append one JSON line per generation of every run to FILE")
    a = ap.parse_args(argv)
    params = dict(variant=a.variant)
    if a.depth:
        params["depth"] = a.depth
    grids = benchmark_instances(a.n, a.r, a.instances)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    if a.mode == "table":
        fh = open(a.log, "a") if a.log else None
        gen_log = (lambda r: (fh.write(json.dumps(r) + "\n"), fh.flush())) if fh else None
        rows = table(grids, a.runs, a.population, a.generations, a.seed, int(a.max_iterations),
                     a.time_limit, log, gen_log, **params)
        if fh:
            fh.close()
        text = _fmt_table(rows)
    else:
        pops = [int(x) for x in a.populations.split(",") if x]
        rows = population_sweep(grids, pops, a.runs, a.generations, a.seed,
                                int(a.max_iterations), a.time_limit, log, **params)
        text = _fmt_sweep(rows)
    if a.json:
        for x in rows:
            print(json.dumps(x))
    else:
        print(f"n={a.n} r={a.r} instances={a.instances} runs={a.runs}")
        print(text)


if __name__ == "__main__":
    main()
