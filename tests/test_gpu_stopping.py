"""GPU path: the iteration budget of Section 4.3, session progress through
plse_peek and the paper-style statistics driver, against the CPU oracle.
Comparisons are exact (integer arithmetic, shared counter-based draws)."""

import sys

import numpy as np
import pytest

from paper_2103_10453_amd import experiments as E
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


# hard: the bound is out of reach, so every generation runs p * depth iterations
HARD = dict(grid=lambda: gen.random_greedy(12, 0.6, 5), p=8, depth=1440, G=6, seed=77)
# individuals finish early: the per-generation counts vary
EASY = dict(grid=lambda: gen.random_greedy(20, 0.5, 7), p=8, depth=4000, G=6, seed=77)


@pytest.mark.parametrize("case,cap", [("hard", 1), ("hard", 11520), ("hard", 11521),
                                      ("hard", 3 * 11520), ("hard", 10 ** 9),
                                      ("easy", 30000), ("easy", 31300)])
def test_iteration_budget_parity(torch_cuda, oracle_mod, case, cap):
    c = HARD if case == "hard" else EASY
    g = c["grid"]()
    _say(f"iteration budget {case} cap={cap}")
    s = P.Solver(g, depth=c["depth"], max_iterations=cap)
    grid, filled = s.solve(c["p"], c["G"], c["seed"])
    st = s.stats()
    I = oracle_mod.Instance(g)
    r = I.run(I.params(depth=c["depth"], max_iterations=cap), c["p"], c["G"], c["seed"])
    assert st["generations_run"] == r["gens"]
    assert filled == r["filled"]
    np.testing.assert_array_equal(grid, r["grid"])
    np.testing.assert_array_equal(st["best_f_per_gen"], r["best_f"][:r["gens"]])
    np.testing.assert_array_equal(st["counters_per_gen"], r["counters"][:r["gens"]])
    spent = int(r["counters"][:r["gens"], 0].sum())
    assert st["stop_reason"] == (E.STOP_BUDGET if spent >= cap else E.STOP_NONE)
    assert int(st["totals"][0]) == spent


def test_peek_reports_each_generation(torch_cuda, oracle_mod):
    """Stepping one generation at a time, plse_peek reports exactly the
    oracle's best f, best generation and cumulative iterations; after the
    budget stops the run, further steps change nothing."""
    c = EASY
    g = c["grid"]()
    I = oracle_mod.Instance(g)
    full = I.run(I.params(depth=c["depth"]), c["p"], c["G"], c["seed"])
    cum = np.cumsum(full["counters"][:, 0].astype(np.int64))
    _say("peek per generation")
    s = P.Solver(g, depth=c["depth"])
    s.begin(c["p"], c["seed"])
    for k in range(1, c["G"] + 1):
        s.step(1)
        pr = s.peek()
        assert pr["generations_run"] == k
        assert pr["best_f"] == full["best_f"][k - 1]
        assert pr["iterations"] == cum[k - 1]
        assert pr["stop_reason"] == 0
        bg = 1 + int(np.argmax(full["best_f"][:k] == full["best_f"][k - 1]))
        assert pr["best_generation"] == bg
    grid, filled = s.end()
    assert filled == full["filled"]
    np.testing.assert_array_equal(grid, full["grid"])

    cap = int(cum[1])
    _say(f"peek after the budget cap={cap}")
    s = P.Solver(g, depth=c["depth"], max_iterations=cap)
    s.begin(c["p"], c["seed"])
    s.step(2)
    pr = s.peek()
    assert (pr["generations_run"], pr["stop_reason"], pr["iterations"]) == (2, E.STOP_BUDGET, cap)
    s.step(3)
    assert s.peek() == pr
    grid, filled = s.end()
    short = I.run(I.params(depth=c["depth"]), c["p"], 2, c["seed"])
    assert filled == short["filled"]
    np.testing.assert_array_equal(grid, short["grid"])


def test_trials_and_summary_equal_independent_solves(torch_cuda, oracle_mod):
    """run_trials: each run equals the oracle run with its seed; the summary
    holds the best and mean score and the oracle's iterations to the best."""
    g = gen.random_greedy(12, 0.6, 5)
    I = oracle_mod.Instance(g)
    _say("experiments.run_trials runs=3")
    recs = []
    tr = E.run_trials(g, runs=3, population=16, generations=4, seed=500, depth=1440,
                      gen_log=recs.append)
    assert len(recs) == 12
    for t in tr:
        r = I.run(I.params(depth=1440), 16, 4, t.seed)
        mine = [x for x in recs if x["seed"] == t.seed]
        assert [x["best_f"] for x in mine] == [int(v) for v in r["best_f"]]
        assert [x["moves"] for x in mine] == [int(v) for v in r["counters"][:, 1]]
        assert all(x["plits_ms"] > 0 for x in mine)
        assert t.filled == r["filled"] and t.generations == r["gens"] == 4
        np.testing.assert_array_equal(t.grid, r["grid"])
        bg = 1 + int(np.argmax(r["best_f"] == r["best_f"][-1]))
        assert t.best_generation == bg
        assert t.iterations_to_best == int(r["counters"][:bg, 0].sum())
        assert t.seconds_to_best > 0 and t.stop_reason == E.STOP_NONE
    sm = E.summarize(tr)
    assert sm["f_best"] == max(t.filled for t in tr)
    assert sm["f_avg"] == pytest.approx(np.mean([t.filled for t in tr]))
    assert sm["optimal"] == (sm["f_best"] == I.ub)


def test_wall_clock_budget_stops_between_generations(torch_cuda, oracle_mod):
    """A zero time limit stops after the first generation; the result is the
    one-generation run's."""
    g = gen.random_greedy(12, 0.6, 5)
    I = oracle_mod.Instance(g)
    _say("experiments time limit 0")
    (t,) = E.run_trials(g, runs=1, population=16, generations=50, seed=9, time_limit_s=0.0,
                        depth=1440)
    assert t.generations == 1 and t.stop_reason == E.STOP_TIME
    r = I.run(I.params(depth=1440), 16, 1, 9)
    assert t.filled == r["filled"]
    np.testing.assert_array_equal(t.grid, r["grid"])


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


def test_served_runs_that_stop_early_leave_at_their_stop(torch_cuda):
    """Served requests stopped by the bound (stop_at_ub) or by their iteration
    budget report the generations actually run and return plse_solve's
    result; a request without a stop runs all its generations beside them."""
    _say("serving: early stops")
    specs = [(gen.planted(10, 0.4, 0), 16, 40, 2, dict(depth=300, stop_at_ub=1)),
             (HARD["grid"](), 8, 6, 77, dict(depth=1440, max_iterations=2 * 11520)),
             (gen.random_greedy(15, 0.4, 21), 24, 3, 5, dict(depth=300))]
    want = []
    for g, p, G, seed, kw in specs:
        s = P.Solver(g, **kw)
        grid, filled = s.solve(p, G, seed)
        want.append((grid, filled, s.stats()["generations_run"]))
    assert want[0][2] < 40 and want[1][2] == 2 and want[2][2] == 3
    srv = P.Server(1 << 30, max_slots=3)
    try:
        tickets = [srv.submit(P.Solver(g, **kw), p, G, seed) for g, p, G, seed, kw in specs]
        res = _wait(srv, tickets)
        for i, t in enumerate(tickets):
            r = res[t]
            assert r["status"] == P.PLSE_OK
            assert r["generations"] == want[i][2]
            assert r["filled"] == want[i][1]
            np.testing.assert_array_equal(r["grid"], want[i][0])
    finally:
        srv.close()


def test_checkpoint_resume_equals_uninterrupted_run(torch_cuda, oracle_mod):
    """A session checkpointed after 2 generations and resumed on a fresh
    handle (its own workspace) for 3 more equals the uninterrupted 5-generation
    run and the oracle's, statistics included; a second checkpoint of the
    resumed session continues the same way; an image of other parameters or
    another population is refused."""
    g = HARD["grid"]()
    p, depth, seed = 24, 1440, 99
    I = oracle_mod.Instance(g)
    full = I.run(I.params(depth=depth), p, 5, seed)
    _say("checkpoint after 2 generations, resume for 3")
    s1 = P.Solver(g, depth=depth)
    s1.begin(p, seed)
    s1.step(2)
    img = s1.checkpoint()
    s1.step(1)
    img3 = s1.checkpoint()
    s1.end()
    s2 = P.Solver(g, depth=depth)
    s2.resume(p, img)
    s2.step(3)
    grid, filled = s2.end()
    st = s2.stats()
    assert filled == full["filled"] and st["generations_run"] == full["gens"] == 5
    np.testing.assert_array_equal(grid, full["grid"])
    np.testing.assert_array_equal(st["best_f_per_gen"], full["best_f"])
    np.testing.assert_array_equal(st["counters_per_gen"], full["counters"])
    assert len(s2.timing()[0]) == 3
    _say("resume from generation 3 on the first handle")
    s1.resume(p, img3)
    s1.step(2)
    grid3, filled3 = s1.end()
    assert filled3 == full["filled"]
    np.testing.assert_array_equal(grid3, full["grid"])
    other = P.Solver(g, depth=depth + 8)
    with pytest.raises(P.PlseError) as e:
        other.resume(p, img)
    assert e.value.status == P.PLSE_E_ARG
    with pytest.raises(P.PlseError) as e:
        s2.resume(p + 2, img)
    assert e.value.status == P.PLSE_E_ARG


def test_server_cancel_waiting_and_resident_requests(torch_cuda):
    """A cancelled waiting request ends without running; a cancelled resident
    one stops at a generation end and returns a legal best grid so far; the
    server keeps serving others, with results equal to plse_solve."""
    import time
    _say("serving: cancellation")
    small = gen.planted(10, 0.4, 0)
    want = P.Solver(small, depth=300).solve(16, 5, 2)
    srv = P.Server(1 << 30, max_slots=1)
    try:
        long = P.Solver(gen.random_greedy(30, 0.5, 3), depth=9000)
        t1 = srv.submit(long, 64, 500, 1)
        t2 = srv.submit(P.Solver(small, depth=300), 16, 5, 2)
        t0 = time.time()
        while srv.status()[1] < 1:
            assert time.time() - t0 < 60
            time.sleep(0.01)
        time.sleep(0.5)
        srv.cancel(t2)
        srv.cancel(t1)
        res = _wait(srv, [t1, t2])
        assert res[t2]["status"] == P.PLSE_E_CANCELLED and res[t2]["generations"] == 0
        r1 = res[t1]
        assert r1["status"] == P.PLSE_E_CANCELLED
        assert 1 <= r1["generations"] < 500
        assert gen.is_partial_latin(r1["grid"]) and 0 < r1["filled"] <= long.ub
        # the statistics cover every generation the request ran, including
        # those still queued when it was cancelled
        st = long.stats()
        assert st["generations_run"] == r1["generations"]
        bf = st["best_f_per_gen"]
        assert len(bf) == r1["generations"] and np.all(np.diff(bf) <= 0)
        assert np.all(st["counters_per_gen"][:, 0] > 0)
        assert long.n * long.n - long.l - int(bf[-1]) == r1["filled"]
        for t in (t1, 12345):
            with pytest.raises(P.PlseError) as e:
                srv.cancel(t)
            assert e.value.status == P.PLSE_E_ARG
        t3 = srv.submit(P.Solver(small, depth=300), 16, 5, 2)
        r3 = _wait(srv, [t3])[t3]
        assert r3["status"] == P.PLSE_OK and r3["filled"] == want[1]
        np.testing.assert_array_equal(r3["grid"], want[0])
    finally:
        srv.close()
