"""plse_solve_noalloc: the allocation-free form of plse_solve (a fixed device
array inside the library instead of an attached workspace) gives exactly the
result and statistics of plse_solve, also on a second, smaller call that
finds the array holding the first call's data."""

import ctypes

import numpy as np
import pytest

from paper_2103_10453_amd import instances as gen
from paper_2103_10453_amd import plse as P


def test_noalloc_rejects_oversized_request_before_device_work():
    # host-only path: the size check comes before any HIP call
    h = P.plse_create(gen.planted(50, 0.5, 1001))
    try:
        with pytest.raises(P.PlseError) as e:
            P.plse_solve_noalloc(h, 50, 16384, 2, 1, stream=0)
        assert e.value.status == P.PLSE_E_CAPACITY
        with pytest.raises(P.PlseError) as e:
            P.plse_solve_noalloc(h, 50, 1, 2, 1, stream=0)
        assert e.value.status == P.PLSE_E_ARG
    finally:
        P.plse_destroy(h)


@pytest.mark.gpu
def test_noalloc_equals_solve_on_two_calls():
    import torch
    torch.cuda.set_device(0)
    cases = [
        (gen.planted(12, 0.4, 71), 96, 4, 11),   # first call: larger
        (gen.random_greedy(9, 0.5, 72), 40, 3, 12),  # second call: smaller instance and population
    ]
    for grid, p, G, seed in cases:
        n = grid.shape[0]
        print(f"noalloc case n={n} p={p} G={G} seed={seed}", flush=True)
        s = P.Solver(grid, depth=10 * n * n)
        ref_grid, ref_filled = s.solve(p, G, seed)
        ref_stats = s.stats()
        g2, f2, need = P.plse_solve_noalloc(s.h, n, p, G, seed)
        torch.cuda.synchronize()
        st = s.stats()
        assert 0 < need <= P.NOALLOC_BYTES
        assert f2 == ref_filled
        assert np.array_equal(g2, ref_grid)
        assert st["generations_run"] == ref_stats["generations_run"]
        assert np.array_equal(st["best_f_per_gen"], ref_stats["best_f_per_gen"])
        assert np.array_equal(st["counters_per_gen"], ref_stats["counters_per_gen"])
        # the attached workspace still serves plse_solve afterwards
        g3, f3 = s.solve(p, G, seed)
        assert f3 == ref_filled and np.array_equal(g3, ref_grid)
