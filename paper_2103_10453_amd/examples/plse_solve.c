/*
 * plse_solve -- extend a partial Latin square from the command line through
 * the C ABI of libplse alone (no Python): the caller owns the device
 * workspace (hipMalloc) and the stream, as include/plse.h asks.
 *
 *   plse_solve POPULATION GENERATIONS SEED [DEPTH] < grid.txt
 *
 * grid.txt: the order n, then n*n symbols row by row (0 = empty, 1..n).
 * Prints the number of filled cells, the upper bound, the generations run
 * and the best grid, in the same format (n, then n rows).  DEPTH (tabu
 * iterations per individual and generation) defaults to 10 n^2.
 * Exit status: 0, or the PLSE_* status of the first failing call (100 + code
 * for a HIP runtime failure of the program itself).
 */
#define __HIP_PLATFORM_AMD__
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "plse.h"

static int fail(const char *what, int status) {
    fprintf(stderr, "%s: %s (status %d)\n", what, plse_strerror(status), status);
    return status;
}

int main(int argc, char **argv) {
    if (argc < 4) {
        fprintf(stderr, "usage: %s POPULATION GENERATIONS SEED [DEPTH] < grid.txt\n", argv[0]);
        return PLSE_E_ARG;
    }
    const int32_t p = (int32_t)atoi(argv[1]), G = (int32_t)atoi(argv[2]);
    const uint64_t seed = strtoull(argv[3], NULL, 10);
    int n = 0;
    if (scanf("%d", &n) != 1 || n < 1 || n > 127) {
        fprintf(stderr, "bad order\n");
        return PLSE_E_ARG;
    }
    int8_t *grid = (int8_t *)malloc((size_t)n * n), *best = (int8_t *)malloc((size_t)n * n);
    for (int c = 0; c < n * n; ++c) {
        int v = 0;
        if (scanf("%d", &v) != 1) {
            fprintf(stderr, "short grid\n");
            return PLSE_E_ARG;
        }
        grid[c] = (int8_t)v;
    }
    plse_handle h = NULL;
    int rc = plse_create(n, grid, &h);
    if (rc) return fail("plse_create", rc);
    if (argc > 4 && (rc = plse_set_param(h, "depth", atoll(argv[4]))) != PLSE_OK)
        return fail("plse_set_param", rc);
    size_t bytes = 0;
    if ((rc = plse_workspace_bytes(h, p, &bytes)) != PLSE_OK) return fail("plse_workspace_bytes", rc);
    void *ws = NULL;
    if (hipMalloc(&ws, bytes) != hipSuccess) return 100 + PLSE_E_HIP;
    if ((rc = plse_attach_workspace(h, ws, bytes)) != PLSE_OK) return fail("plse_attach_workspace", rc);
    hipStream_t stream = NULL;
    if (hipStreamCreate(&stream) != hipSuccess) return 100 + PLSE_E_HIP;
    int32_t filled = 0;
    if ((rc = plse_solve(h, p, G, seed, stream, best, &filled)) != PLSE_OK)
        return fail("plse_solve", rc);
    int32_t nv = 0, l = 0, ub = 0;
    plse_info(h, &nv, &l, &ub);
    plse_stats st;
    plse_last_stats(h, &st, NULL, NULL);
    printf("filled %d bound %d generations %d\n", filled, ub, st.generations_run);
    printf("%d\n", n);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) printf("%d%c", best[r * n + c], c + 1 < n ? ' ' : '\n');
    plse_attach_workspace(h, NULL, 0);
    plse_destroy(h);
    (void)hipStreamDestroy(stream);
    (void)hipFree(ws);
    free(grid);
    free(best);
    return 0;
}
