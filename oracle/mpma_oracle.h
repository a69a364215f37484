/*
 * mpma_oracle.h -- CPU oracle of the MPMA hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct CPU
 * implementation of what the GPU path computes, written from Goudet & Hao,
 * "A massively parallel evolutionary algorithm for the partial Latin square
 * extension problem".  It shares no code with the GPU library.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Every function follows the passage it cites; where the paper is silent the
 * documented reading is taken (random streams, tie-breaks, phase split, ...).
 * All arithmetic is integer.
 *
 * Parity status of each part (what pins it, see tests/test_oracle_*.py):
 *   orc_create     Alg. 1 + upper bound: worked n=3 example, planted l=0,
 *                  brute-force UB on tiny grids.
 *   philox / fmix  Random123 known-answer vectors; fmix32 inverted exactly.
 *   orc_init       invariants: legal, maximal, prefilled kept.
 *   orc_plits      from-scratch recomputation after every move (paranoid
 *                  mode) and an independent brute-force re-derivation of every
 *                  move on tiny instances.  Partial-MPMA's PartialCol: the
 *                  same recomputation check, legality after every search,
 *                  and f never above the repaired offspring's.
 *   orc_distances  numpy broadcast definition.
 *   orc_select     literal transcription of Alg. 4 (with the documented
 *                  termination/fill fix).
 *   orc_match      numpy masked argmin; random matching (Section 5.3): never
 *                  the individual itself, uniform over the others.
 *   orc_aux        closed-form expected distances of Section 3.5.2; UX keeps
 *                  half the differing positions (binomial bound); no
 *                  crossover copies the first parent exactly.
 *   counters       every counter of a search re-derived from the brute-force
 *                  move trace (iterations, moves, idle, candidates, eligible
 *                  vertices, neighbour and count updates, snapshots).
 *   orc_run        a literal transcription of Alg. 2 (tests/refdefs.py) on
 *                  tiny grids: final population, f, uids, partner
 *                  histories, offspring, S* and best f per generation equal;
 *                  planted slips in the bookkeeping (history dropped, uids
 *                  by rank, transposed distances, first offspring) fail it.
 *                  filled <= UB; planted instances complete; brute-force
 *                  optimum on tiny grids; with an iteration cap, the stop
 *                  generation is the first whose cumulative count reaches the
 *                  cap (fixed per-generation count on a hard instance) and the
 *                  capped run is a prefix of the uncapped one.
 *   AUX threshold  exact big-integer Eq. 9 threshold, also where
 *                  (beta D - |V|) 2^32 exceeds 64 bits.
 */
#ifndef MPMA_ORACLE_H
#define MPMA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameter vector (int64) indices. */
enum {
    ORC_P_DEPTH1 = 0,   /* phase-1 iterations  (Section 3.3: 100|V| by default) */
    ORC_P_DEPTH2,       /* phase-2 iterations  (Section 3.3: 2|V|)              */
    ORC_P_ALPHA_NUM,    /* tabu tenure alpha = num/den = 6/10                    */
    ORC_P_ALPHA_DEN,
    ORC_P_BETA_NUM,     /* AUX beta = num/den = 20/1 (Eq. 9)                     */
    ORC_P_BETA_DEN,
    ORC_P_SPACING,      /* gamma of Section 3.4 = 10                             */
    ORC_P_STOP_AT_UB,   /* 1: stop after the generation that reaches the bound   */
    ORC_P_HIST,         /* partner-history length (<= ORC_HMAX)                  */
    ORC_P_PARANOID,     /* 1: recompute the state from scratch after each move   */
    ORC_P_CROSSOVER,    /* ORC_X_*: AUX (Alg. 5), UX or none (Section 5.2)       */
    ORC_P_MATCHING,     /* ORC_M_*: nearest neighbour (3.5.1) or random (5.3)    */
    ORC_P_VARIANT,      /* ORC_V_*: MPMA or Partial-MPMA (Section 3.7)           */
    ORC_P_MAX_ITERS,    /* > 0: stop after the generation whose cumulative tabu  */
                        /* iterations (whole population) reach this cap (the     */
                        /* iteration budget of Section 4.3); 0: no cap           */
    ORC_NPARAMS
};

#define ORC_HMAX 64

/* Crossover variants (Section 3.5.2, Section 5.2). */
enum { ORC_X_AUX = 0, ORC_X_UX = 1, ORC_X_NONE = 2 };
/* Parent matching variants (Section 3.5.1, Section 5.3). */
enum { ORC_M_NEAREST = 0, ORC_M_RANDOM = 1 };
/* Algorithm variants: MPMA, or Partial-MPMA (Section 3.7: repaired offspring
 * and the PartialCol tabu search over legal partial colourings). */
enum { ORC_V_MPMA = 0, ORC_V_PARTIAL = 1 };

/* Counter vector indices (per individual, summed over phases). */
enum {
    ORC_C_ITERS = 0,    /* iterations with a non-empty eligible set              */
    ORC_C_MOVES,        /* iterations that applied a move                        */
    ORC_C_IDLE,         /* iterations with no admissible candidate               */
    ORC_C_CANDS,        /* candidate one-moves examined                          */
    ORC_C_ELIG,         /* eligible vertices, summed over iterations             */
    ORC_C_NUPD,         /* conflict-table entries updated by moves: the          */
                        /* incremental evaluation of Section 3.3 changes         */
                        /* conf[u][old] and conf[u][new] of every neighbour u    */
                        /* of the moved vertex, one entry per coloured end       */
    ORC_C_SNAPS,        /* best-solution snapshots                               */
    ORC_C_REPAIRS,      /* vertices uncoloured by the final repair               */
    ORC_C_CUPD,         /* row/column colour counts changed by moves (2 per      */
                        /* coloured end: the factored form of the same table,    */
                        /* conf[v][k] = row count + column count - 2[S(v) = k])  */
    ORC_NCOUNTERS
};

/* Returns a handle or NULL; *status = 0 ok, 1 bad argument, 2 bad grid. */
void *orc_create(int32_t n, const int8_t *grid, int32_t *status);
void  orc_destroy(void *h);
/* out[0]=|V|, out[1]=l, out[2]=UB, out[3]=sum |D*(v)| */
void  orc_info(const void *h, int32_t out[4]);
/* Export the reduced graph: vertex row/col, domain CSR (offsets |V|+1). */
void  orc_tables(const void *h, int32_t *vrow, int32_t *vcol, int32_t *dom_off, uint8_t *dom);

void  orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t orc_fmix32(uint32_t x);
/* Tie value of move (v, k) under tie words wv, wk (best-move ties, Section 3.3). */
uint32_t orc_tie16(uint32_t wv, uint32_t wk, uint32_t v, uint32_t k);

/* Randomised greedy legal initial colourings of slots 0..p-1. */
void orc_init(const void *h, uint64_t seed, int32_t p, uint8_t *S, int32_t *f);
/* The same for the listed slots only (row i of S is slot slots[i]). */
void orc_init_slots(const void *h, uint64_t seed, int32_t ns, const int32_t *slots, uint8_t *S,
                    int32_t *f);

/* PLITS on `ns` individuals; slot ids key the random streams.
 * S_in/S_out: ns*|V| colours.  counters: ns*ORC_NCOUNTERS. */
void orc_plits(const void *h, const int64_t *params, uint64_t seed, int32_t gen,
               int32_t ns, const int32_t *slots, const uint8_t *S_in,
               uint8_t *S_out, int32_t *f_out, uint64_t *counters);

/* Move trace of one PLITS run (tiny instances): per iteration
 * {phase, it, v, k, delta, F_after, idle}; returns the number of rows. */
int32_t orc_plits_trace(const void *h, const int64_t *params, uint64_t seed, int32_t gen,
                        int32_t slot, const uint8_t *S_in, int32_t max_rows, int64_t *rows);

/* D[i*nb+j] = Hamming distance between A_i and B_j (Eq. 8). */
void orc_distances(int32_t nv, int32_t na, const uint8_t *A, int32_t nb, const uint8_t *B,
                   int32_t *D);

/* Population update (Alg. 4) over P^all (2p candidates, D_all 2p*2p). */
void orc_select(int32_t nv, int32_t p, int64_t spacing, uint64_t seed, int32_t gen,
                const int32_t *f_all, const int32_t *D_all, int32_t *accepted);

/* Nearest-neighbour matching with partner history (Section 3.5.1). */
void orc_match(int32_t p, const int32_t *D, const uint64_t *uid, uint64_t *hist,
               int32_t *hcount, int32_t hlen, int32_t *partner, int32_t *dpart);
/* The same with a matching variant (ORC_M_*); random matching draws from
 * (seed, slot i, generation gen). */
void orc_match_mode(int32_t p, const int32_t *D, const uint64_t *uid, uint64_t *hist,
                    int32_t *hcount, int32_t hlen, int32_t mode, uint64_t seed, int32_t gen,
                    int32_t *partner, int32_t *dpart);

/* AUX crossover (Alg. 5, Eq. 9). */
void orc_aux(int32_t nv, int32_t p, uint64_t seed, int32_t gen, int64_t beta_num,
             int64_t beta_den, const uint8_t *S, const int32_t *partner,
             const int32_t *dpart, uint8_t *S_off);
/* The same with a crossover variant (ORC_X_*). */
void orc_aux_mode(int32_t nv, int32_t p, uint64_t seed, int32_t gen, int64_t beta_num,
                  int64_t beta_den, int32_t mode, const uint8_t *S, const int32_t *partner,
                  const int32_t *dpart, uint8_t *S_off);

/* Whole MPMA run (Alg. 2).  best_f_gen[G], counters_gen[G*ORC_NCOUNTERS]
 * (zero past the last generation run).  final_S (p*|V|) may be NULL.
 * Returns the number of generations run, or <0 on error. */
int32_t orc_run(const void *h, const int64_t *params, int32_t p, int32_t G, uint64_t seed,
                int8_t *grid_out, int32_t *filled, int32_t *best_f_gen,
                uint64_t *counters_gen, uint8_t *final_S, int32_t *final_f);

/* State of Alg. 2 after a run, for comparison at a generation boundary: the
 * uids, partner histories (ring of ORC_HMAX, write position hcount % hlen,
 * see orc_match) and their counts of the final population, the offspring
 * waiting for the next search (p*|V|) and S* (|V|).  Any pointer may be
 * NULL.  After an early stop (bound or budget) the population is the one
 * the stopping generation started from. */
typedef struct {
    uint64_t *uid;
    uint64_t *hist;
    int32_t *hcount;
    uint8_t *offspring;
    uint8_t *best;
} orc_state_t;
int32_t orc_run_state(const void *h, const int64_t *params, int32_t p, int32_t G, uint64_t seed,
                      int8_t *grid_out, int32_t *filled, int32_t *best_f_gen,
                      uint64_t *counters_gen, uint8_t *final_S, int32_t *final_f,
                      const orc_state_t *state);

/* AUX threshold of Eq. 9 on a 32-bit draw: floor((beta D - |V|) 2^32 /
 * (beta D)) with beta = beta_num / beta_den, 0 when beta D <= |V|. */
uint64_t orc_aux_threshold(int64_t beta_num, int64_t beta_den, int32_t D, int32_t nv);

#ifdef __cplusplus
}
#endif
#endif
