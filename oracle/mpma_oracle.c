/*
 * mpma_oracle.c -- CPU oracle of the MPMA hot path (test infrastructure only).
 *
 * Plain C, dense tables, no blocking or incremental tricks beyond what the
 * paper itself states (the conflict table of the "streamline" evaluation,
 * Section 3.3).  Written from the paper; shares nothing with the GPU library.
 * See mpma_oracle.h for the list of pins that tie each function to the paper.
 */
#include "mpma_oracle.h"

#include <limits.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Counter-based randomness.                                                 */
/* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11.  Ten rounds of two 32x32->64 multiplies with a   */
/* Weyl-sequence key schedule.                                               */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* MurmurHash3 32-bit finaliser (Appleby): a bijection on 32-bit words. */
uint32_t orc_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

/* Tie value of move (v, k) in an iteration with tie words wv, wk: the top
 * 16 bits of fmix32(wv ^ v) ^ fmix32(wk ^ k).  Both words are fresh every
 * iteration, so the colours of one vertex, and one colour over several
 * vertices, are ordered at random each time. */
uint32_t orc_tie16(uint32_t wv, uint32_t wk, uint32_t v, uint32_t k) {
    return (orc_fmix32(wv ^ v) ^ orc_fmix32(wk ^ k)) >> 16;
}

/* Stream tags: which random decision a draw belongs to. */
#define TAG_INIT_ORDER 0x01u
#define TAG_INIT_PICK  0x02u
#define TAG_PLITS1     0x11u
#define TAG_PLITS2     0x12u
#define TAG_PARTIAL    0x13u
#define TAG_SELECT     0x21u
#define TAG_XOVER      0x31u
#define TAG_MATCH      0x41u

/* Counter = (instance key 0, slot, gen<<8 | tag, index); key = seed halves. */
static void draw(uint64_t seed, uint32_t slot, uint32_t gen, uint32_t tag, uint32_t idx,
                 uint32_t out[4]) {
    uint32_t ctr[4] = {0u, slot, (gen << 8) | tag, idx};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* Uniform integer in [0, m): floor(w * m / 2^32). */
static uint32_t scale(uint32_t w, uint32_t m) { return (uint32_t)(((uint64_t)w * m) >> 32); }

/* ------------------------------------------------------------------------ */
/* Instance: Latin square graph (Section 2.1) reduced by Alg. 1 (Section 2.2) */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n, nv, l, ub, nd;
    int8_t *grid;      /* n*n copy of the input                              */
    int *cell_v;       /* n*n: vertex id, -1 prefilled, -2 impossible       */
    int *vrow, *vcol;  /* nv                                                 */
    int *dom_off;      /* nv+1: D*(v) in dom[dom_off[v] .. dom_off[v+1])     */
    uint8_t *dom;      /* nd colours, ascending                              */
    uint8_t *in_dom;   /* nv*(n+1): 1 iff colour k is in D*(v)               */
    int *row_v, *row_cnt; /* vertices of each row    (n*n, n)                */
    int *col_v, *col_cnt; /* vertices of each column (n*n, n)                */
} inst_t;

void *orc_create(int32_t n, const int8_t *grid, int32_t *status) {
    *status = 0;
    if (n < 1 || n > 127 || grid == NULL) { *status = 1; return NULL; }
    /* A partial Latin square: symbols in [0, n], none repeated in a row or
     * column (Section 1). */
    for (int i = 0; i < n * n; i++)
        if (grid[i] < 0 || grid[i] > n) { *status = 2; return NULL; }
    for (int r = 0; r < n; r++)
        for (int a = 0; a < n; a++)
            for (int b = a + 1; b < n; b++) {
                int8_t x = grid[r * n + a], y = grid[r * n + b];
                if (x && x == y) { *status = 2; return NULL; }
                x = grid[a * n + r]; y = grid[b * n + r];
                if (x && x == y) { *status = 2; return NULL; }
            }

    inst_t *I = (inst_t *)calloc(1, sizeof(inst_t));
    I->n = n;
    I->grid = (int8_t *)malloc((size_t)n * n);
    memcpy(I->grid, grid, (size_t)n * n);
    I->cell_v = (int *)malloc(sizeof(int) * n * n);

    /* Alg. 1: every prefilled cell removes its symbol from the domains of the
     * empty cells in its row and column; an empty cell left with D = {0} is
     * impossible (counted in l) and removed.  Removing a prefilled vertex
     * never changes another prefilled one, so one pass suffices. */
    uint8_t *dstar = (uint8_t *)calloc((size_t)n * n * (n + 1), 1); /* dstar[cell][k] */
    int nv = 0, nd = 0, l = 0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            int c = i * n + j;
            if (grid[c] != 0) { I->cell_v[c] = -1; continue; }
            int cnt = 0;
            for (int k = 1; k <= n; k++) {
                int used = 0;
                for (int t = 0; t < n; t++)
                    if (grid[i * n + t] == k || grid[t * n + j] == k) used = 1;
                if (!used) { dstar[(size_t)c * (n + 1) + k] = 1; cnt++; }
            }
            if (cnt == 0) { I->cell_v[c] = -2; l++; }
            else { I->cell_v[c] = nv++; nd += cnt; }
        }
    I->nv = nv; I->nd = nd; I->l = l;
    /* Upper bound (Section 2.2): n^2 - l, or n^2 - 2 when l = 1. */
    I->ub = (l == 1) ? n * n - 2 : n * n - l;

    I->vrow = (int *)malloc(sizeof(int) * (nv + 1));
    I->vcol = (int *)malloc(sizeof(int) * (nv + 1));
    I->dom_off = (int *)malloc(sizeof(int) * (nv + 1));
    I->dom = (uint8_t *)malloc((size_t)nd + 1);
    I->in_dom = (uint8_t *)calloc((size_t)(nv + 1) * (n + 1), 1);
    I->row_v = (int *)malloc(sizeof(int) * n * n);
    I->col_v = (int *)malloc(sizeof(int) * n * n);
    I->row_cnt = (int *)calloc(n, sizeof(int));
    I->col_cnt = (int *)calloc(n, sizeof(int));
    int pos = 0;
    for (int c = 0; c < n * n; c++) {
        int v = I->cell_v[c];
        if (v < 0) continue;
        int i = c / n, j = c % n;
        I->vrow[v] = i; I->vcol[v] = j;
        I->dom_off[v] = pos;
        for (int k = 1; k <= n; k++)
            if (dstar[(size_t)c * (n + 1) + k]) {
                I->dom[pos++] = (uint8_t)k;
                I->in_dom[(size_t)v * (n + 1) + k] = 1;
            }
        I->row_v[i * n + I->row_cnt[i]++] = v;
        I->col_v[j * n + I->col_cnt[j]++] = v;
    }
    I->dom_off[nv] = pos;
    free(dstar);
    return I;
}

void orc_destroy(void *h) {
    inst_t *I = (inst_t *)h;
    if (!I) return;
    free(I->grid); free(I->cell_v); free(I->vrow); free(I->vcol); free(I->dom_off);
    free(I->dom); free(I->in_dom); free(I->row_v); free(I->col_v); free(I->row_cnt);
    free(I->col_cnt); free(I);
}

void orc_info(const void *h, int32_t out[4]) {
    const inst_t *I = (const inst_t *)h;
    out[0] = I->nv; out[1] = I->l; out[2] = I->ub; out[3] = I->nd;
}

void orc_tables(const void *h, int32_t *vrow, int32_t *vcol, int32_t *dom_off, uint8_t *dom) {
    const inst_t *I = (const inst_t *)h;
    for (int v = 0; v < I->nv; v++) { vrow[v] = I->vrow[v]; vcol[v] = I->vcol[v]; }
    for (int v = 0; v <= I->nv; v++) dom_off[v] = I->dom_off[v];
    memcpy(dom, I->dom, (size_t)I->nd);
}

/* Neighbours of v in the reduced graph: the other vertices of its row and of
 * its column (Section 2.1).  Calls fn(u) for each. */
#define FOR_NEIGHBOURS(I, v, u, BODY)                                          \
    do {                                                                        \
        int r_ = (I)->vrow[v], c_ = (I)->vcol[v];                               \
        for (int t_ = 0; t_ < (I)->row_cnt[r_]; t_++) {                         \
            int u = (I)->row_v[r_ * (I)->n + t_];                               \
            if (u != (v)) { BODY; }                                             \
        }                                                                       \
        for (int t_ = 0; t_ < (I)->col_cnt[c_]; t_++) {                         \
            int u = (I)->col_v[c_ * (I)->n + t_];                               \
            if (u != (v)) { BODY; }                                             \
        }                                                                       \
    } while (0)

/* ------------------------------------------------------------------------ */
/* Initial population (Alg. 2 initialisation, Section 3.2).  Reading: a     */
/* randomised greedy legal colouring -- vertices visited in the order of     */
/* their INIT_ORDER draws (ties by id), each given a uniformly drawn colour  */
/* among those of D*(v) not used by an already coloured neighbour, or left   */
/* uncoloured if none is left.                                              */
/* ------------------------------------------------------------------------ */
static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static void init_one(const inst_t *I, uint64_t seed, uint32_t slot, uint8_t *S) {
    int n = I->n, nv = I->nv;
    uint64_t *order = (uint64_t *)malloc(sizeof(uint64_t) * (nv + 1));
    for (int v = 0; v < nv; v++) {
        uint32_t w[4];
        draw(seed, slot, 0, TAG_INIT_ORDER, (uint32_t)v >> 2, w);
        order[v] = ((uint64_t)w[v & 3] << 32) | (uint32_t)v;
    }
    qsort(order, (size_t)nv, sizeof(uint64_t), cmp_u64);
    uint8_t *row_used = (uint8_t *)calloc((size_t)n * (n + 1), 1);
    uint8_t *col_used = (uint8_t *)calloc((size_t)n * (n + 1), 1);
    uint8_t *legal = (uint8_t *)malloc((size_t)n + 1);
    memset(S, 0, (size_t)nv);
    for (int t = 0; t < nv; t++) {
        int v = (int)(uint32_t)order[t];
        int r = I->vrow[v], c = I->vcol[v], cnt = 0;
        for (int q = I->dom_off[v]; q < I->dom_off[v + 1]; q++) {
            int k = I->dom[q];
            if (!row_used[r * (n + 1) + k] && !col_used[c * (n + 1) + k]) legal[cnt++] = (uint8_t)k;
        }
        if (cnt == 0) continue;
        uint32_t w[4];
        draw(seed, slot, 0, TAG_INIT_PICK, (uint32_t)t, w);
        int k = legal[scale(w[0], (uint32_t)cnt)];
        S[v] = (uint8_t)k;
        row_used[r * (n + 1) + k] = 1;
        col_used[c * (n + 1) + k] = 1;
    }
    free(order); free(row_used); free(col_used); free(legal);
}

static int count_uncoloured(const uint8_t *S, int nv) {
    int f = 0;
    for (int v = 0; v < nv; v++) f += (S[v] == 0);
    return f;
}

void orc_init(const void *h, uint64_t seed, int32_t p, uint8_t *S, int32_t *f) {
    const inst_t *I = (const inst_t *)h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < p; i++) {
        init_one(I, seed, (uint32_t)i, S + (size_t)i * I->nv);
        f[i] = count_uncoloured(S + (size_t)i * I->nv, I->nv);
    }
}

void orc_init_slots(const void *h, uint64_t seed, int32_t ns, const int32_t *slots, uint8_t *S,
                    int32_t *f) {
    const inst_t *I = (const inst_t *)h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < ns; i++) {
        init_one(I, seed, (uint32_t)slots[i], S + (size_t)i * I->nv);
        f[i] = count_uncoloured(S + (size_t)i * I->nv, I->nv);
    }
}

/* ------------------------------------------------------------------------ */
/* PLITS: two-phase tabu search (Section 3.3, Alg. 3).                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int *conf;      /* nv*(n+1): conf[v][k] = #neighbours of v coloured k     */
    int64_t *tabu;  /* nv*(n+1): iteration from which move (v,k) is allowed   */
    uint8_t *best;  /* nv                                                      */
} work_t;

/* conf, f, c of S from scratch (Eq. 1, Eq. 3). */
static void full_state(const inst_t *I, const uint8_t *S, int *conf, int64_t *f, int64_t *c) {
    int n = I->n, nv = I->nv;
    memset(conf, 0, sizeof(int) * (size_t)nv * (n + 1));
    for (int v = 0; v < nv; v++) {
        FOR_NEIGHBOURS(I, v, u, { if (S[u]) conf[(size_t)v * (n + 1) + S[u]]++; });
    }
    int64_t ff = 0, cc2 = 0;
    for (int v = 0; v < nv; v++) {
        if (S[v] == 0) ff++;
        else cc2 += conf[(size_t)v * (n + 1) + S[v]];
    }
    *f = ff;
    *c = cc2 / 2; /* every conflicting edge is seen from both ends */
}

static int eligible(const inst_t *I, const uint8_t *S, const int *conf, int v) {
    /* V_0 or C(S): uncoloured, or coloured and sharing its colour with a
     * neighbour (Section 3.3). */
    return S[v] == 0 || conf[(size_t)v * (I->n + 1) + S[v]] > 0;
}

static void die_if(int cond) {
    if (cond) abort();
}

/* One phase.  S is updated in place to the phase's best solution. */
static void plits_phase(const inst_t *I, const int64_t *P, uint64_t seed, uint32_t slot,
                        uint32_t gen, int phase, int64_t iters, uint8_t *S, work_t *W,
                        uint64_t *cnt, int64_t *trace, int32_t *trace_rows, int32_t trace_max) {
    int n = I->n, nv = I->nv;
    /* Extended fitness F = f + phi*c (Eq. 6) kept as phi_den*F:
     * phase 1 phi = 1/2, phase 2 phi = |V| (Section 3.3). */
    int64_t phi_num = (phase == 1) ? 1 : nv;
    int64_t phi_den = (phase == 1) ? 2 : 1;
    uint32_t tag = (phase == 1) ? TAG_PLITS1 : TAG_PLITS2;
    int64_t f, c;
    full_state(I, S, W->conf, &f, &c);
    int64_t F = phi_den * f + phi_num * c;
    int64_t Fbest = F;
    memcpy(W->best, S, (size_t)nv);
    for (size_t q = 0; q < (size_t)nv * (n + 1); q++) W->tabu[q] = 0;

    for (int64_t it = 0; it < iters; it++) {
        int m = 0;
        for (int v = 0; v < nv; v++) m += eligible(I, S, W->conf, v);
        if (m == 0) break; /* F = 0: nothing left to improve */
        cnt[ORC_C_ITERS]++;
        cnt[ORC_C_ELIG] += (uint64_t)m;
        uint32_t w[4];
        draw(seed, slot, gen, tag, (uint32_t)it, w);

        /* Best admissible one-move of N(S) = N_0(S) u N_c(S) (Eq. 7). */
        uint64_t best_key = UINT64_MAX;
        int bv = -1, bk = -1;
        int64_t bdelta = 0;
        for (int v = 0; v < nv; v++) {
            if (!eligible(I, S, W->conf, v)) continue;
            int s = S[v];
            int cur = s ? W->conf[(size_t)v * (n + 1) + s] : 0;
            /* candidate colours: D(v) = {0} u D*(v), minus the current one;
             * an uncoloured vertex only moves to D*(v). */
            for (int q = I->dom_off[v] - 1; q < I->dom_off[v + 1]; q++) {
                int k = (q < I->dom_off[v]) ? 0 : I->dom[q];
                if (k == s) continue;
                cnt[ORC_C_CANDS]++;
                int64_t df = (s == 0 ? -1 : 0) + (k == 0 ? 1 : 0);
                int64_t dc = (k ? W->conf[(size_t)v * (n + 1) + k] : 0) - cur;
                int64_t delta = phi_den * df + phi_num * dc;
                /* admissible: not tabu, or better than the phase's best
                 * (aspiration). */
                int adm = (it >= W->tabu[(size_t)v * (n + 1) + k]) || (F + delta < Fbest);
                if (!adm) continue;
                /* ties: smaller tie value t(v, k) first, then smaller move
                 * id v(n+1)+k; the scan visits ids in increasing order, so
                 * a strict comparison of (delta, t) keeps the smallest id. */
                uint32_t t = orc_tie16(w[1], w[2], (uint32_t)v, (uint32_t)k);
                uint64_t key = ((uint64_t)(uint32_t)(delta + 0x80000000LL) << 32) | t;
                if (key < best_key) { best_key = key; bv = v; bk = k; bdelta = delta; }
            }
        }
        if (bv < 0) {
            cnt[ORC_C_IDLE]++;
            if (trace && *trace_rows < trace_max) {
                int64_t *row = trace + 7 * (*trace_rows)++;
                row[0] = phase; row[1] = it; row[2] = -1; row[3] = -1; row[4] = 0;
                row[5] = F; row[6] = 1;
            }
            continue;
        }

        /* Apply: move bv from its colour class to class bk. */
        int old = S[bv];
        int64_t dc = (bk ? W->conf[(size_t)bv * (n + 1) + bk] : 0) -
                     (old ? W->conf[(size_t)bv * (n + 1) + old] : 0);
        FOR_NEIGHBOURS(I, bv, u, {
            if (old) W->conf[(size_t)u * (n + 1) + old]--;
            if (bk) W->conf[(size_t)u * (n + 1) + bk]++;
        });
        /* work counters: the conflict-table entries of every neighbour, for
         * the colour left and for the colour taken; and, in the factored form
         * of the table, the row and column counts of those two colours */
        {
            uint64_t deg = 0;
            FOR_NEIGHBOURS(I, bv, u, { (void)u; deg++; });
            cnt[ORC_C_NUPD] += deg * (uint64_t)((old != 0) + (bk != 0));
        }
        cnt[ORC_C_CUPD] += 2u * (old != 0) + 2u * (bk != 0);
        S[bv] = (uint8_t)bk;
        f += (bk == 0) - (old == 0);
        c += dc;
        F += bdelta;
        die_if(F != phi_den * f + phi_num * c);
        if (P[ORC_P_PARANOID]) {
            int64_t f2, c2;
            int *conf2 = (int *)malloc(sizeof(int) * (size_t)nv * (n + 1));
            full_state(I, S, conf2, &f2, &c2);
            die_if(f2 != f || c2 != c);
            for (int v = 0; v < nv; v++)
                for (int q = I->dom_off[v]; q < I->dom_off[v + 1]; q++)
                    die_if(conf2[(size_t)v * (n + 1) + I->dom[q]] !=
                           W->conf[(size_t)v * (n + 1) + I->dom[q]]);
            free(conf2);
        }

        /* Tabu tenure T = L + alpha*(|V_0| + |C(S)|), L uniform in [0, 9],
         * counted after the move; the reverse move (bv back to `old`) is
         * forbidden for the next T iterations. */
        int mp = 0;
        for (int v = 0; v < nv; v++) mp += eligible(I, S, W->conf, v);
        int64_t T = (int64_t)scale(w[0], 10u) + (P[ORC_P_ALPHA_NUM] * mp) / P[ORC_P_ALPHA_DEN];
        W->tabu[(size_t)bv * (n + 1) + old] = it + 1 + T;
        cnt[ORC_C_MOVES]++;

        if (F < Fbest) {
            Fbest = F;
            memcpy(W->best, S, (size_t)nv);
            cnt[ORC_C_SNAPS]++;
        }
        if (trace && *trace_rows < trace_max) {
            int64_t *row = trace + 7 * (*trace_rows)++;
            row[0] = phase; row[1] = it; row[2] = bv; row[3] = bk; row[4] = bdelta;
            row[5] = F; row[6] = 0;
        }
    }
    memcpy(S, W->best, (size_t)nv);
}

/* Greedy conflict removal (Section 3.7): uncolour the vertex with the most
 * conflicts first (ties: lowest id) until the colouring is legal. */
static void repair(const inst_t *I, uint8_t *S, int *conf, uint64_t *cnt) {
    int n = I->n, nv = I->nv;
    int64_t f, c;
    full_state(I, S, conf, &f, &c);
    for (;;) {
        int bv = -1, bc = 0;
        for (int v = 0; v < nv; v++)
            if (S[v] && conf[(size_t)v * (n + 1) + S[v]] > bc) {
                bc = conf[(size_t)v * (n + 1) + S[v]];
                bv = v;
            }
        if (bv < 0) break;
        int old = S[bv];
        FOR_NEIGHBOURS(I, bv, u, { conf[(size_t)u * (n + 1) + old]--; });
        S[bv] = 0;
        cnt[ORC_C_REPAIRS]++;
    }
}

/* PartialCol (Section 3.7, the legal-colouring tabu search of Partial-MPMA,
 * adapted to list colouring).  S is a legal partial colouring and stays one;
 * the search minimises f = |V_0|.  A move gives an uncoloured vertex v a
 * colour k of D*(v) and uncolours the neighbours of v that hold k (Delta f =
 * their number - 1); those neighbours may not take k again for T iterations
 * unless that reaches a better f than the search's best (aspiration).  Best
 * move, ties, tenure T = L + alpha |V_0| (after the move) and the snapshot of
 * the best solution follow the conventions of the two-phase search.  S is
 * updated in place to the best solution found. */
static void partialcol(const inst_t *I, const int64_t *P, uint64_t seed, uint32_t slot,
                       uint32_t gen, int64_t iters, uint8_t *S, work_t *W, uint64_t *cnt) {
    int n = I->n, nv = I->nv;
    int64_t f, c;
    full_state(I, S, W->conf, &f, &c);
    die_if(c != 0);
    int64_t fbest = f;
    memcpy(W->best, S, (size_t)nv);
    for (size_t q = 0; q < (size_t)nv * (n + 1); q++) W->tabu[q] = 0;
    int *gone = (int *)malloc(sizeof(int) * (size_t)(2 * n + 2));

    for (int64_t it = 0; it < iters; it++) {
        if (f == 0) break; /* complete: nothing left to colour */
        cnt[ORC_C_ITERS]++;
        cnt[ORC_C_ELIG] += (uint64_t)f;
        uint32_t w[4];
        draw(seed, slot, gen, TAG_PARTIAL, (uint32_t)it, w);
        uint64_t best_key = UINT64_MAX;
        int bv = -1, bk = -1;
        int64_t bdelta = 0;
        for (int v = 0; v < nv; v++) {
            if (S[v] != 0) continue;
            for (int q = I->dom_off[v]; q < I->dom_off[v + 1]; q++) {
                int k = I->dom[q];
                cnt[ORC_C_CANDS]++;
                int64_t delta = (int64_t)W->conf[(size_t)v * (n + 1) + k] - 1;
                int adm = (it >= W->tabu[(size_t)v * (n + 1) + k]) || (f + delta < fbest);
                if (!adm) continue;
                uint32_t t = orc_tie16(w[1], w[2], (uint32_t)v, (uint32_t)k);
                uint64_t key = ((uint64_t)(uint32_t)(delta + 0x80000000LL) << 32) | t;
                if (key < best_key) { best_key = key; bv = v; bk = k; bdelta = delta; }
            }
        }
        if (bv < 0) {
            cnt[ORC_C_IDLE]++;
            continue;
        }
        /* bv joins class bk; its neighbours in class bk leave it */
        int ng = 0;
        uint64_t upd = 0;
        FOR_NEIGHBOURS(I, bv, u, {
            if (S[u] == bk) gone[ng++] = u;
            W->conf[(size_t)u * (n + 1) + bk]++;
            upd++;
        });
        S[bv] = (uint8_t)bk;
        for (int q = 0; q < ng; q++) {
            int u = gone[q];
            S[u] = 0;
            FOR_NEIGHBOURS(I, u, x, { W->conf[(size_t)x * (n + 1) + bk]--; upd++; });
        }
        die_if(ng - 1 != bdelta);
        f += bdelta;
        cnt[ORC_C_NUPD] += upd;
        cnt[ORC_C_CUPD] += 2u + 2u * (uint64_t)ng;
        if (P[ORC_P_PARANOID]) {
            int64_t f2, c2;
            int *conf2 = (int *)malloc(sizeof(int) * (size_t)nv * (n + 1));
            full_state(I, S, conf2, &f2, &c2);
            die_if(f2 != f || c2 != 0);
            for (int v = 0; v < nv; v++)
                for (int q = I->dom_off[v]; q < I->dom_off[v + 1]; q++)
                    die_if(conf2[(size_t)v * (n + 1) + I->dom[q]] !=
                           W->conf[(size_t)v * (n + 1) + I->dom[q]]);
            free(conf2);
        }
        int64_t T = (int64_t)scale(w[0], 10u) + (P[ORC_P_ALPHA_NUM] * f) / P[ORC_P_ALPHA_DEN];
        for (int q = 0; q < ng; q++) W->tabu[(size_t)gone[q] * (n + 1) + bk] = it + 1 + T;
        cnt[ORC_C_MOVES]++;
        if (f < fbest) {
            fbest = f;
            memcpy(W->best, S, (size_t)nv);
            cnt[ORC_C_SNAPS]++;
        }
    }
    free(gone);
    memcpy(S, W->best, (size_t)nv);
}

static void phase_lengths(const int64_t *P, int64_t *i1, int64_t *i2) {
    *i1 = P[ORC_P_DEPTH1];
    *i2 = P[ORC_P_DEPTH2];
}

static void plits_one(const inst_t *I, const int64_t *P, uint64_t seed, uint32_t gen,
                      uint32_t slot, const uint8_t *S_in, uint8_t *S_out, int32_t *f_out,
                      uint64_t *cnt, int64_t *trace, int32_t *trace_rows, int32_t trace_max) {
    int n = I->n, nv = I->nv;
    work_t W;
    W.conf = (int *)malloc(sizeof(int) * (size_t)(nv + 1) * (n + 1));
    W.tabu = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv + 1) * (n + 1));
    W.best = (uint8_t *)malloc((size_t)nv + 1);
    int64_t i1, i2;
    phase_lengths(P, &i1, &i2);
    memcpy(S_out, S_in, (size_t)nv);
    for (int q = 0; q < ORC_NCOUNTERS; q++) cnt[q] = 0;
    if (P[ORC_P_VARIANT] == ORC_V_PARTIAL) {
        /* Partial-MPMA (Section 3.7): the offspring is repaired into a legal
         * partial colouring, then improved by PartialCol for the whole depth */
        repair(I, S_out, W.conf, cnt);
        partialcol(I, P, seed, slot, gen, i1 + i2, S_out, &W, cnt);
    } else {
        /* Phase 1 explores with phi = 1/2; phase 2 starts from phase 1's best
         * and drives conflicts out with phi = |V| (Section 3.3). */
        plits_phase(I, P, seed, slot, gen, 1, i1, S_out, &W, cnt, trace, trace_rows, trace_max);
        plits_phase(I, P, seed, slot, gen, 2, i2, S_out, &W, cnt, trace, trace_rows, trace_max);
        repair(I, S_out, W.conf, cnt);
    }
    *f_out = count_uncoloured(S_out, nv);
    free(W.conf); free(W.tabu); free(W.best);
}

void orc_plits(const void *h, const int64_t *params, uint64_t seed, int32_t gen, int32_t ns,
               const int32_t *slots, const uint8_t *S_in, uint8_t *S_out, int32_t *f_out,
               uint64_t *counters) {
    const inst_t *I = (const inst_t *)h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < ns; i++) {
        int32_t rows = 0;
        plits_one(I, params, seed, (uint32_t)gen, (uint32_t)slots[i], S_in + (size_t)i * I->nv,
                  S_out + (size_t)i * I->nv, f_out + i, counters + (size_t)i * ORC_NCOUNTERS,
                  NULL, &rows, 0);
    }
}

int32_t orc_plits_trace(const void *h, const int64_t *params, uint64_t seed, int32_t gen,
                        int32_t slot, const uint8_t *S_in, int32_t max_rows, int64_t *rows) {
    const inst_t *I = (const inst_t *)h;
    uint8_t *S_out = (uint8_t *)malloc((size_t)I->nv + 1);
    uint64_t cnt[ORC_NCOUNTERS];
    int32_t f, nrows = 0;
    plits_one(I, params, seed, (uint32_t)gen, (uint32_t)slot, S_in, S_out, &f, cnt, rows, &nrows,
              max_rows);
    free(S_out);
    return nrows;
}

/* ------------------------------------------------------------------------ */
/* Hamming distance (Eq. 8).                                                 */
/* ------------------------------------------------------------------------ */
void orc_distances(int32_t nv, int32_t na, const uint8_t *A, int32_t nb, const uint8_t *B,
                   int32_t *D) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < na; i++)
        for (int j = 0; j < nb; j++) {
            int d = 0;
            for (int v = 0; v < nv; v++) d += (A[(size_t)i * nv + v] != B[(size_t)j * nv + v]);
            D[(size_t)i * nb + j] = d;
        }
}

/* ------------------------------------------------------------------------ */
/* Population update (Alg. 4).  P^all = P_t (0..p-1) u P' (p..2p-1).        */
/* Candidates are examined best first -- by f, then by a SELECT draw, then  */
/* by index -- and each is examined once: it joins P_{t+1} when the         */
/* population is not full and spacing*D > |V| to every member already in.   */
/* If the scan ends short of p members, rejected candidates are appended in */
/* scan order.                                                              */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t f; uint32_t w; int32_t x; } selkey_t;

static int cmp_selkey(const void *a, const void *b) {
    const selkey_t *x = (const selkey_t *)a, *y = (const selkey_t *)b;
    if (x->f != y->f) return (x->f > y->f) - (x->f < y->f);
    if (x->w != y->w) return (x->w > y->w) - (x->w < y->w);
    return (x->x > y->x) - (x->x < y->x);
}

void orc_select(int32_t nv, int32_t p, int64_t spacing, uint64_t seed, int32_t gen,
                const int32_t *f_all, const int32_t *D_all, int32_t *accepted) {
    int m = 2 * p;
    selkey_t *k = (selkey_t *)malloc(sizeof(selkey_t) * m);
    for (int x = 0; x < m; x++) {
        uint32_t w[4];
        draw(seed, 0, (uint32_t)gen, TAG_SELECT, (uint32_t)x >> 2, w);
        k[x].f = f_all[x]; k[x].w = w[x & 3]; k[x].x = x;
    }
    qsort(k, (size_t)m, sizeof(selkey_t), cmp_selkey);
    int32_t *rejected = (int32_t *)malloc(sizeof(int32_t) * m);
    int na = 0, nr = 0;
    for (int r = 0; r < m; r++) {
        int x = k[r].x, ok = (na < p);
        for (int a = 0; ok && a < na; a++)
            if (!(spacing * (int64_t)D_all[(size_t)x * m + accepted[a]] > nv)) ok = 0;
        if (ok) accepted[na++] = x;
        else rejected[nr++] = x;
    }
    for (int r = 0; na < p; r++) accepted[na++] = rejected[r];
    free(k); free(rejected);
}

/* ------------------------------------------------------------------------ */
/* Parent matching (Section 3.5.1): the second parent of S_i is its nearest */
/* neighbour (ties: lowest slot) among the individuals it has not yet been  */
/* crossed with; if all are excluded, the plain nearest neighbour.          */
/* ------------------------------------------------------------------------ */
void orc_match_mode(int32_t p, const int32_t *D, const uint64_t *uid, uint64_t *hist,
                    int32_t *hcount, int32_t hlen, int32_t mode, uint64_t seed, int32_t gen,
                    int32_t *partner, int32_t *dpart) {
    for (int i = 0; i < p; i++) {
        int best = -1;
        if (mode == ORC_M_RANDOM) {
            /* Section 5.3: the second parent is drawn uniformly among the
             * other p - 1 individuals. */
            uint32_t w[4];
            draw(seed, (uint32_t)i, (uint32_t)gen, TAG_MATCH, 0u, w);
            best = (int)scale(w[0], (uint32_t)(p - 1));
            if (best >= i) best++;
        }
        for (int pass = 0; pass < 2 && best < 0; pass++)
            for (int j = 0; j < p; j++) {
                if (j == i) continue;
                if (pass == 0) {
                    int seen = 0;
                    for (int t = 0; t < hcount[i] && t < hlen; t++)
                        if (hist[(size_t)i * ORC_HMAX + t] == uid[j]) seen = 1;
                    if (seen) continue;
                }
                if (best < 0 || D[(size_t)i * p + j] < D[(size_t)i * p + best]) best = j;
            }
        partner[i] = best;
        dpart[i] = D[(size_t)i * p + best];
        /* remember this crossover: FIFO of the last `hlen` partners */
        if (hlen > 0) {
            int pos = hcount[i] % hlen;
            hist[(size_t)i * ORC_HMAX + pos] = uid[best];
            hcount[i]++;
            if (hcount[i] >= 2 * hlen) hcount[i] -= hlen; /* keep the write position, stay full */
        }
    }
}

void orc_match(int32_t p, const int32_t *D, const uint64_t *uid, uint64_t *hist,
               int32_t *hcount, int32_t hlen, int32_t *partner, int32_t *dpart) {
    orc_match_mode(p, D, uid, hist, hcount, hlen, ORC_M_NEAREST, 0, 0, partner, dpart);
}

/* ------------------------------------------------------------------------ */
/* AUX crossover (Alg. 5): vertex v inherits S_i(v) with probability        */
/* p_ij = 1 - |V| / (beta * D_ij) (Eq. 9), else S_j(v).  The probability is */
/* the integer threshold floor((beta*D - |V|) * 2^32 / (beta*D)) on a 32-bit */
/* draw, and 0 when beta*D <= |V|.                                          */
/* ------------------------------------------------------------------------ */
uint64_t orc_aux_threshold(int64_t beta_num, int64_t beta_den, int32_t D, int32_t nv) {
    /* p_ij = 1 - |V| / (beta D) = (beta_num D - beta_den |V|) / (beta_num D),
     * scaled by 2^32; the numerator times 2^32 needs more than 64 bits for
     * large beta terms, so the division is done in 128 bits */
    uint64_t bd = (uint64_t)beta_num * (uint64_t)D;
    uint64_t bv = (uint64_t)beta_den * (uint64_t)nv;
    if (bd <= bv) return 0;
    return (uint64_t)((((unsigned __int128)(bd - bv)) << 32) / bd);
}

void orc_aux_mode(int32_t nv, int32_t p, uint64_t seed, int32_t gen, int64_t beta_num,
                  int64_t beta_den, int32_t mode, const uint8_t *S, const int32_t *partner,
                  const int32_t *dpart, uint8_t *S_off) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < p; i++) {
        int j = partner[i];
        uint64_t thr = orc_aux_threshold(beta_num, beta_den, dpart[i], nv);
        /* UX: p_ij fixed at 1/2 (Section 3.5.2); no crossover: the offspring
         * is a copy of its first parent (Section 5.2) */
        if (mode == ORC_X_UX) thr = 1ull << 31;
        if (mode == ORC_X_NONE) thr = 1ull << 32;
        for (int v = 0; v < nv; v++) {
            uint32_t w[4];
            draw(seed, (uint32_t)i, (uint32_t)gen, TAG_XOVER, (uint32_t)v >> 2, w);
            S_off[(size_t)i * nv + v] =
                ((uint64_t)w[v & 3] < thr) ? S[(size_t)i * nv + v] : S[(size_t)j * nv + v];
        }
    }
}

void orc_aux(int32_t nv, int32_t p, uint64_t seed, int32_t gen, int64_t beta_num,
             int64_t beta_den, const uint8_t *S, const int32_t *partner, const int32_t *dpart,
             uint8_t *S_off) {
    orc_aux_mode(nv, p, seed, gen, beta_num, beta_den, ORC_X_AUX, S, partner, dpart, S_off);
}

/* ------------------------------------------------------------------------ */
/* Whole run (Alg. 2).                                                      */
/* ------------------------------------------------------------------------ */
int32_t orc_run(const void *h, const int64_t *P, int32_t p, int32_t G, uint64_t seed,
                int8_t *grid_out, int32_t *filled, int32_t *best_f_gen,
                uint64_t *counters_gen, uint8_t *final_S, int32_t *final_f) {
    return orc_run_state(h, P, p, G, seed, grid_out, filled, best_f_gen, counters_gen, final_S,
                         final_f, NULL);
}

int32_t orc_run_state(const void *h, const int64_t *P, int32_t p, int32_t G, uint64_t seed,
                      int8_t *grid_out, int32_t *filled, int32_t *best_f_gen,
                      uint64_t *counters_gen, uint8_t *final_S, int32_t *final_f,
                      const orc_state_t *state) {
    const inst_t *I = (const inst_t *)h;
    int n = I->n, nv = I->nv, m = 2 * p;
    if (p < 2 || G < 1) return -1;
    size_t snv = (size_t)nv;
    uint8_t *Sall = (uint8_t *)calloc((size_t)m * snv + 1, 1); /* P_t then P' */
    uint8_t *Snext = (uint8_t *)calloc((size_t)p * snv + 1, 1);
    uint8_t *Soff = (uint8_t *)calloc((size_t)p * snv + 1, 1);
    uint8_t *Sstar = (uint8_t *)calloc(snv + 1, 1);
    int32_t *fall = (int32_t *)calloc(m, sizeof(int32_t));
    int32_t *fnext = (int32_t *)calloc(p, sizeof(int32_t));
    uint64_t *uid = (uint64_t *)calloc(m, sizeof(uint64_t));
    uint64_t *uidn = (uint64_t *)calloc(p, sizeof(uint64_t));
    uint64_t *hist = (uint64_t *)calloc((size_t)m * ORC_HMAX, sizeof(uint64_t));
    uint64_t *histn = (uint64_t *)calloc((size_t)p * ORC_HMAX, sizeof(uint64_t));
    int32_t *hc = (int32_t *)calloc(m, sizeof(int32_t));
    int32_t *hcn = (int32_t *)calloc(p, sizeof(int32_t));
    int32_t *Dall = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * m);
    int32_t *Dn = (int32_t *)malloc(sizeof(int32_t) * (size_t)p * p);
    int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * p);
    int32_t *partner = (int32_t *)malloc(sizeof(int32_t) * p);
    int32_t *dpart = (int32_t *)malloc(sizeof(int32_t) * p);
    int32_t *slots = (int32_t *)malloc(sizeof(int32_t) * p);
    uint64_t *cnt = (uint64_t *)calloc((size_t)p * ORC_NCOUNTERS, sizeof(uint64_t));
    int hlen = (int)P[ORC_P_HIST];
    if (hlen > ORC_HMAX) hlen = ORC_HMAX;

    /* P_1 = initial population; its first offspring population is itself. */
    orc_init(h, seed, p, Sall, fall);
    for (int i = 0; i < p; i++) { uid[i] = (uint64_t)i; slots[i] = i; }
    memcpy(Soff, Sall, (size_t)p * snv);

    int32_t fstar = INT32_MAX, gens = 0;
    uint64_t iters_total = 0;
    for (int g = 1; g <= G; g++) {
        gens = g;
        /* local search on every offspring, in parallel */
        orc_plits(h, P, seed, g, p, slots, Soff, Sall + (size_t)p * snv, fall + p, cnt);
        for (int q = 0; q < ORC_NCOUNTERS; q++) {
            uint64_t s = 0;
            for (int i = 0; i < p; i++) s += cnt[(size_t)i * ORC_NCOUNTERS + q];
            counters_gen[(size_t)(g - 1) * ORC_NCOUNTERS + q] = s;
        }
        /* best solution saving */
        int b = 0;
        for (int i = 1; i < p; i++)
            if (fall[p + i] < fall[p + b]) b = i;
        if (fall[p + b] < fstar) {
            fstar = fall[p + b];
            memcpy(Sstar, Sall + (size_t)(p + b) * snv, snv);
        }
        best_f_gen[g - 1] = fstar;
        if (P[ORC_P_STOP_AT_UB] && n * n - I->l - fstar == I->ub) break;
        /* iteration budget (Section 4.3): checked once per generation */
        iters_total += counters_gen[(size_t)(g - 1) * ORC_NCOUNTERS + 0];
        if (P[ORC_P_MAX_ITERS] > 0 && iters_total >= (uint64_t)P[ORC_P_MAX_ITERS]) break;

        /* distances over P^all, population update, new uids */
        orc_distances(nv, m, Sall, m, Sall, Dall);
        orc_select(nv, p, P[ORC_P_SPACING], seed, g, fall, Dall, acc);
        for (int i = 0; i < p; i++) { uid[p + i] = ((uint64_t)g << 32) | (uint32_t)i; hc[p + i] = 0; }
        for (int r = 0; r < p; r++) {
            int x = acc[r];
            memcpy(Snext + (size_t)r * snv, Sall + (size_t)x * snv, snv);
            fnext[r] = fall[x];
            uidn[r] = uid[x];
            hcn[r] = hc[x];
            memcpy(histn + (size_t)r * ORC_HMAX, hist + (size_t)x * ORC_HMAX,
                   sizeof(uint64_t) * ORC_HMAX);
        }
        for (int i = 0; i < p; i++)
            for (int j = 0; j < p; j++) Dn[(size_t)i * p + j] = Dall[(size_t)acc[i] * m + acc[j]];
        memcpy(Sall, Snext, (size_t)p * snv);
        memcpy(fall, fnext, sizeof(int32_t) * p);
        memcpy(uid, uidn, sizeof(uint64_t) * p);
        memcpy(hc, hcn, sizeof(int32_t) * p);
        memcpy(hist, histn, sizeof(uint64_t) * (size_t)p * ORC_HMAX);

        /* parent matching and AUX offspring for the next generation */
        orc_match_mode(p, Dn, uid, hist, hc, hlen, (int32_t)P[ORC_P_MATCHING], seed, g, partner,
                       dpart);
        orc_aux_mode(nv, p, seed, g, P[ORC_P_BETA_NUM], P[ORC_P_BETA_DEN],
                     (int32_t)P[ORC_P_CROSSOVER], Sall, partner, dpart, Soff);
    }
    for (int g = gens; g < G; g++) {
        best_f_gen[g] = fstar;
        for (int q = 0; q < ORC_NCOUNTERS; q++) counters_gen[(size_t)g * ORC_NCOUNTERS + q] = 0;
    }

    /* best grid: prefilled cells, then S* on the vertices */
    for (int c = 0; c < n * n; c++) {
        int v = I->cell_v[c];
        grid_out[c] = (v == -1) ? I->grid[c] : (v >= 0 ? (int8_t)Sstar[v] : 0);
    }
    int fl = 0;
    for (int c = 0; c < n * n; c++) fl += (grid_out[c] != 0);
    *filled = fl;
    if (final_S) memcpy(final_S, Sall, (size_t)p * snv);
    if (final_f) memcpy(final_f, fall, sizeof(int32_t) * p);
    if (state) {
        if (state->uid) memcpy(state->uid, uid, sizeof(uint64_t) * p);
        if (state->hist) memcpy(state->hist, hist, sizeof(uint64_t) * (size_t)p * ORC_HMAX);
        if (state->hcount) memcpy(state->hcount, hc, sizeof(int32_t) * p);
        if (state->offspring) memcpy(state->offspring, Soff, (size_t)p * snv);
        if (state->best) memcpy(state->best, Sstar, snv);
    }

    free(Sall); free(Snext); free(Soff); free(Sstar); free(fall); free(fnext); free(uid);
    free(uidn); free(hist); free(histn); free(hc); free(hcn); free(Dall); free(Dn); free(acc);
    free(partner); free(dpart); free(slots); free(cnt);
    return gens;
}
