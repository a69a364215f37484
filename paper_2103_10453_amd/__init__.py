"""MI355X (gfx950) solver for the partial Latin square extension problem.

The hot path of Goudet & Hao's massively parallel memetic algorithm (tabu
search, distances, population update, parent matching, AUX crossover) runs in
the HIP kernels of libplse.so behind the C ABI of include/plse.h; `plse` is
its Python binding and `instances` the seeded input generators.
"""
