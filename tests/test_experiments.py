"""Host-side statistics of the paper-style driver (no GPU): records built
from per-generation statistics, the per-instance summary of Tables 3-4 and
Appendix A, and the population-sweep aggregation of Section 5.1."""

import numpy as np
import pytest

from paper_2103_10453_amd import experiments as E
from paper_2103_10453_amd import instances as gen


def _stats(iters, best_gen, gens=None):
    cnt = np.zeros((len(iters), 9), dtype=np.uint64)
    cnt[:, 0] = iters
    return dict(generations_run=gens if gens is not None else len(iters),
                best_generation=best_gen, counters_per_gen=cnt)


def test_trial_record_counts_up_to_the_best_generation():
    st = _stats([10, 20, 30, 40], 2)
    t = E.trial_record(5, 99, 100, st, [1.0, 2.0, 3.0, 4.0], [0.5, 0.5, 0.5, 0.5], 1.25, 0)
    assert (t.iterations, t.iterations_to_best) == (100, 30)
    assert t.seconds_to_best == pytest.approx((1.0 + 0.5 + 2.0 + 0.5) / 1e3)
    assert (t.generations, t.best_generation, t.filled, t.upper_bound) == (4, 2, 99, 100)
    # no generation run: nothing to the best
    t0 = E.trial_record(5, 0, 100, _stats([], 0), [], [], 0.1, 0)
    assert (t0.iterations, t0.iterations_to_best, t0.seconds_to_best) == (0, 0, 0.0)


def test_summary_columns():
    mk = lambda f, it, ts: E.Trial(seed=0, filled=f, upper_bound=12, generations=3,
                                   best_generation=1, iterations=100, iterations_to_best=it,
                                   seconds=1.0, seconds_to_best=ts, stop_reason=0)
    sm = E.summarize([mk(10, 40, 1.0), mk(12, 60, 3.0), mk(11, 20, 2.0)])
    assert (sm["f_best"], sm["runs"], sm["optimal"]) == (12, 3, True)
    assert sm["f_avg"] == pytest.approx(11.0)
    assert sm["nb_iter"] == pytest.approx(40.0) and sm["t_best_s"] == pytest.approx(2.0)
    assert E.summarize([mk(10, 1, 1.0)])["optimal"] is False
    with pytest.raises(ValueError):
        E.summarize([])


def test_population_sweep_aggregation(monkeypatch):
    rows = {
        16: [dict(f_best=10, f_avg=9.0, nb_iter=5.0, t_best_s=1.0),
             dict(f_best=20, f_avg=20.0, nb_iter=7.0, t_best_s=3.0)],
        64: [dict(f_best=11, f_avg=10.0, nb_iter=9.0, t_best_s=2.0),
             dict(f_best=20, f_avg=19.0, nb_iter=3.0, t_best_s=4.0)],
    }
    monkeypatch.setattr(E, "table", lambda grids, runs, p, *a, **k: rows[p])
    out = E.population_sweep([None, None], [16, 64], runs=2)
    assert [x["population"] for x in out] == [16, 64]
    assert out[0]["f_avg"] == pytest.approx(14.5) and out[1]["f_avg"] == pytest.approx(14.5)
    assert out[0]["f_best"] == pytest.approx(15.0) and out[1]["f_best"] == pytest.approx(15.5)
    # best per instance over all sizes: 11 and 20
    assert (out[0]["reach_best"], out[1]["reach_best"]) == (1, 2)
    assert out[1]["nb_iter"] == pytest.approx(6.0)


def test_benchmark_instances_shape_and_seeds():
    a = E.benchmark_instances(20, 0.6, 3)
    b = E.benchmark_instances(20, 0.6, 3)
    assert len(a) == 3
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
        assert gen.is_partial_latin(x)
        assert x.shape == (20, 20)
    assert not np.array_equal(a[0], a[1])


def test_generation_records():
    st = _stats([10, 20, 30], 2)
    st["best_f_per_gen"] = np.array([5, 3, 3], dtype=np.int32)
    st["counters_per_gen"][:, 1] = [9, 18, 27]
    recs = E.generation_records(st, [1.0, 2.0], [0.5, 0.25], 100, 2)  # resumed: 2 timed
    assert [r["generation"] for r in recs] == [1, 2, 3]
    assert [r["score"] for r in recs] == [93, 95, 95]
    assert [r["iterations"] for r in recs] == [10, 20, 30]
    assert [r["moves"] for r in recs] == [9, 18, 27]
    assert recs[0]["plits_ms"] is None and recs[1]["plits_ms"] == 1.0 and recs[2]["rest_ms"] == 0.25
