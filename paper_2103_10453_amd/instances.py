"""Seeded synthetic PLSE instances (input generators only).

This module builds partial Latin squares of the shapes the paper evaluates on
(orders n in {50, 60, 70}, prefill ratios r in 0.3..0.8, Section 4.1) and the
small planted cases used for parity tests.  It holds none of the solver's
arithmetic: it only produces grids.  Both the CPU oracle tests and the GPU
path read their inputs from here.

Randomness comes from splitmix64 (Steele, Lea and Flood, OOPSLA 2014), a
64-bit counter hash that is stable across Python and numpy versions.

Grids are numpy int8 arrays of shape (n, n): 0 = empty, 1..n = symbol.
"""

from __future__ import annotations

import numpy as np

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64 stream: state += golden gamma, then a 3-step finaliser."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def below(self, m: int) -> int:
        """Uniform integer in [0, m) by rejection (exactly uniform)."""
        if m <= 0:
            raise ValueError("m must be positive")
        limit = (1 << 64) - ((1 << 64) % m)
        while True:
            x = self.next_u64()
            if x < limit:
                return x % m

    def permutation(self, m: int) -> list[int]:
        """Fisher-Yates shuffle of range(m)."""
        a = list(range(m))
        for i in range(m - 1, 0, -1):
            j = self.below(i + 1)
            a[i], a[j] = a[j], a[i]
        return a

    def uniform01(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def planted(n: int, prefill: float, seed: int) -> np.ndarray:
    """Planted instance: a permuted cyclic Latin square with cells blanked.

    L[i][j] = (i + j) mod n, then rows, columns and symbols are permuted by
    seeded Fisher-Yates shuffles and symbols shifted to 1..n.  Exactly
    round((1 - prefill) * n^2) cells are blanked: the first cells of a seeded
    permutation of the n^2 cells.  The full square is a completion, so the
    optimum fills all n^2 cells (Section 2.1: the LSC case).
    """
    if n < 1 or n > 127:
        raise ValueError("n must be in [1, 127]")
    rng = SplitMix64(seed)
    prow = rng.permutation(n)
    pcol = rng.permutation(n)
    psym = rng.permutation(n)
    g = np.zeros((n, n), dtype=np.int8)
    for i in range(n):
        for j in range(n):
            g[i, j] = psym[(prow[i] + pcol[j]) % n] + 1
    nblank = int(round((1.0 - prefill) * n * n))
    cells = rng.permutation(n * n)
    for c in cells[:nblank]:
        g[c // n, c % n] = 0
    return g


def random_greedy(n: int, prefill: float, seed: int) -> np.ndarray:
    """Non-planted instance built as the paper's benchmark set was (Section 4.1).

    Cells are visited in a seeded random order; each gets a symbol chosen
    uniformly among those still legal in its row and column (cells with none
    are skipped) until round(prefill * n^2) cells are filled.  The optimum is
    unknown in general.
    """
    if n < 1 or n > 127:
        raise ValueError("n must be in [1, 127]")
    rng = SplitMix64(seed)
    target = int(round(prefill * n * n))
    g = np.zeros((n, n), dtype=np.int8)
    row_used = [set() for _ in range(n)]
    col_used = [set() for _ in range(n)]
    filled = 0
    for c in rng.permutation(n * n):
        if filled >= target:
            break
        i, j = c // n, c % n
        legal = [k for k in range(1, n + 1) if k not in row_used[i] and k not in col_used[j]]
        if not legal:
            continue
        k = legal[rng.below(len(legal))]
        g[i, j] = k
        row_used[i].add(k)
        col_used[j].add(k)
        filled += 1
    return g


def is_partial_latin(grid: np.ndarray) -> bool:
    """True iff every row and column holds each non-zero symbol at most once."""
    g = np.asarray(grid)
    n = g.shape[0]
    if g.shape != (n, n) or g.min() < 0 or g.max() > n:
        return False
    for axis_view in (g, g.T):
        for line in axis_view:
            nz = line[line != 0]
            if len(np.unique(nz)) != len(nz):
                return False
    return True


# ---------------------------------------------------------------------------
# Named workloads.  Instance seed s_k = 1000 * config + k; solver seed is
# s_k + 2^32.  These stand in for the paper's benchmark instances (Haraguchi
# 2016, Section 4.1), which are not available here.
# ---------------------------------------------------------------------------

def solver_seed(instance_seed: int) -> int:
    return instance_seed + (1 << 32)


def workload_small(k: int = 0):
    """Planted n=10, 40% prefilled: population 64, 20 generations, depth 10 n^2."""
    s = 1000 * 0 + k
    return dict(grid=planted(10, 0.4, s), seed=solver_seed(s), population=64,
                generations=20, depth=10 * 10 * 10)


def workload_n50(k: int = 0):
    """Planted n=50, 50% prefilled: population 16384, 50 generations, depth 10 n^2."""
    s = 1000 * 1 + k
    return dict(grid=planted(50, 0.5, s), seed=solver_seed(s), population=16384,
                generations=50, depth=10 * 50 * 50)


def workload_n70(prefill: float, k: int = 0):
    """Random-greedy n=70 at prefill 0.3 / 0.5 / 0.7: population 16384, 100 generations."""
    s = 1000 * 2 + k + int(round(prefill * 100)) * 10
    return dict(grid=random_greedy(70, prefill, s), seed=solver_seed(s), population=16384,
                generations=100, depth=10 * 70 * 70)


def workload_batch(count: int = 256, base: int = 3000):
    """Batch of instances: n ~ U{20..70}, r ~ U[0.3, 0.7] rounded to 0.01,
    first half planted, second half random-greedy; population 1024, 50 generations."""
    out = []
    meta = SplitMix64(base)
    for k in range(count):
        n = 20 + meta.below(51)
        r = round(0.3 + 0.4 * meta.uniform01(), 2)
        s = base + k
        g = planted(n, r, s) if k < count // 2 else random_greedy(n, r, s)
        out.append(dict(grid=g, seed=solver_seed(s), population=1024, generations=50,
                        depth=10 * n * n))
    return out


def workload_served(count: int, rate: float, base: int = 4000):
    """Poisson request stream: exponential gaps at `rate` req/s, n ~ U{10..100},
    r ~ U[0.3, 0.7], planted or random-greedy by coin flip; population 2048,
    50 generations.  Returns a list of dicts with an `arrival` time in seconds.
    The requests and the order of their gaps do not depend on the rate: a
    stream at another rate is the same stream with its gaps rescaled."""
    meta = SplitMix64(base)
    t = 0.0
    out = []
    for k in range(count):
        u = meta.uniform01()
        t += -np.log(1.0 - u) / rate
        n = 10 + meta.below(91)
        r = round(0.3 + 0.4 * meta.uniform01(), 2)
        s = base + k
        g = planted(n, r, s) if meta.below(2) == 0 else random_greedy(n, r, s)
        out.append(dict(grid=g, seed=solver_seed(s), population=2048, generations=50,
                        depth=10 * n * n, arrival=t))
    return out
