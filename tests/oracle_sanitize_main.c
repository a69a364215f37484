/*
 * Driver of the CPU oracle for a sanitizer build (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only): whole runs of MPMA and
 * Partial-MPMA and every crossover / matching variant on small grids, plus
 * the paranoid recomputation mode.  Exit status 0 when every run ends and
 * stays within its bound; the sanitizers abort on any memory or undefined-
 * behaviour error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpma_oracle.h"

/* A cyclic Latin square of order n with every k-th cell blanked. */
static void make_grid(int n, int k, int8_t *g) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) g[i * n + j] = (int8_t)(((i + j) % n) + 1);
    for (int c = 0; c < n * n; c += k) g[c] = 0;
    for (int c = 1; c < n * n; c += 2 * k + 1) g[c] = 0;
}

int main(void) {
    const int sizes[3][2] = {{6, 2}, {9, 3}, {12, 2}};
    int8_t grid[144], out[144];
    for (int t = 0; t < 3; ++t) {
        const int n = sizes[t][0];
        make_grid(n, sizes[t][1], grid);
        int32_t st = 0;
        void *h = orc_create(n, grid, &st);
        if (!h) {
            fprintf(stderr, "orc_create failed %d\n", st);
            return 1;
        }
        for (int variant = 0; variant < 6; ++variant) {
            int64_t P[ORC_NPARAMS];
            memset(P, 0, sizeof(P));
            P[ORC_P_DEPTH1] = 8 * n * n;
            P[ORC_P_DEPTH2] = 2 * n * n;
            P[ORC_P_ALPHA_NUM] = 6;
            P[ORC_P_ALPHA_DEN] = 10;
            P[ORC_P_BETA_NUM] = 20;
            P[ORC_P_BETA_DEN] = 1;
            P[ORC_P_SPACING] = 10;
            P[ORC_P_HIST] = 8;
            P[ORC_P_PARANOID] = variant == 0;
            P[ORC_P_CROSSOVER] = variant % 3;
            P[ORC_P_MATCHING] = variant == 4;
            P[ORC_P_VARIANT] = variant == 5;
            P[ORC_P_MAX_ITERS] = variant == 3 ? 3000 : 0;
            const int p = 8, G = 3;
            int32_t filled = 0, bf[3];
            uint64_t cnt[3 * ORC_NCOUNTERS];
            const int32_t gens = orc_run(h, P, p, G, 7 + variant, out, &filled, bf, cnt, NULL, NULL);
            if (gens < 1 || filled > n * n) {
                fprintf(stderr, "run n=%d variant=%d: gens %d filled %d\n", n, variant, gens, filled);
                return 1;
            }
        }
        orc_destroy(h);
    }
    printf("oracle sanitizer runs ok\n");
    return 0;
}
