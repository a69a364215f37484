/*
 * plse.h -- C ABI of the MI355X (gfx950) solver for the partial Latin square
 * extension problem, after Goudet & Hao, "A massively parallel evolutionary
 * algorithm for the partial Latin square extension problem".
 *
 * Every call returns an int status (PLSE_OK = 0) and never throws.  There is
 * no global state: everything lives in a handle.  The library never allocates
 * device memory: the caller attaches a workspace (e.g. a torch uint8 tensor)
 * and passes a HIP stream; all device work is enqueued on that stream.
 *
 * Threading: one call at a time per handle (PLSE_E_BUSY otherwise).
 */
#ifndef PLSE_H
#define PLSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PLSE_OK = 0,
    PLSE_E_ARG = 1,        /* null pointer or argument out of range             */
    PLSE_E_GRID = 2,       /* grid is not a partial Latin square                */
    PLSE_E_WORKSPACE = 3,  /* no workspace attached, or too small               */
    PLSE_E_HIP = 4,        /* a HIP runtime call failed (see plse_strerror)     */
    PLSE_E_BUSY = 5,       /* the handle is already running a call              */
    PLSE_PENDING = 6,      /* server: request not finished yet                  */
    PLSE_E_PARAM = 7,      /* unknown parameter key or value out of range       */
    PLSE_E_CAPACITY = 8,   /* server: request cannot ever fit the budget        */
    PLSE_E_FAULT = 9,      /* server: request ended by the fault-injection hook */
    PLSE_E_CANCELLED = 10  /* server: request cancelled (plse_server_cancel)    */
};

typedef struct plse_instance *plse_handle;

/* Number of per-generation counters reported by plse_last_stats and the
 * per-individual counter rows of plse_stage_plits, in this order:
 * iterations, moves, idle iterations, candidates examined, eligible vertices
 * (summed over iterations), conflict-table entries updated (the incremental
 * evaluation of Section 3.3 changes the entries of every neighbour of the
 * moved vertex, once per coloured end), best-solution snapshots, vertices
 * uncoloured by the final repair, row/column colour counts updated (the
 * factored form of the same table this library keeps: two per coloured
 * end). */
#define PLSE_NCOUNTERS 9
#define PLSE_MAX_GENERATIONS 65536
#define PLSE_MAX_POPULATION 32768
#define PLSE_HIST 64

typedef struct {
    int32_t generations_run;      /* <= requested generations (UB stop)         */
    int32_t best_f;               /* uncoloured vertices of S*                  */
    int32_t best_generation;      /* generation in which S* was found           */
    int32_t stop_reason;          /* 0 all generations run, 1 bound reached     */
                                  /* (stop_at_ub), 2 iteration budget spent     */
    uint64_t totals[PLSE_NCOUNTERS];
} plse_stats;

/*
 * plse_create -- build the reduced Latin square graph of one instance.
 *
 * Section 2.1 (Latin square graph, list colouring with D(v)) and Alg. 1 of
 * Section 2.2 (preprocessing): prefilled cells are removed and their symbols
 * deleted from the domains of the empty cells in the same row and column; an
 * empty cell left with no symbol is impossible and counted in l.  The upper
 * bound is n^2 - l, or n^2 - 2 when l = 1 (Section 2.2).
 *
 * n:    order, 1..127.
 * grid: host pointer, n*n int8 row-major; 0 = empty, 1..n = symbol.  Copied.
 * out:  receives the handle (free with plse_destroy).
 * Errors: PLSE_E_ARG (null, n out of range), PLSE_E_GRID (a value outside
 * [0, n] or a symbol repeated in a row or column).
 */
int plse_create(int32_t n, const int8_t *grid, plse_handle *out);

/* Section 2.2 and Alg. 1: |V| (empty cells with a non-empty domain, the
 * vertices of the reduced graph), l (empty cells whose domain is empty: they
 * stay empty in every extension) and the upper bound on the score of
 * Section 2.2, n^2 - l, or n^2 - 2 when l = 1.  Host-only; errors:
 * PLSE_E_ARG (null). */
int plse_info(plse_handle h, int32_t *num_vertices, int32_t *num_impossible,
              int32_t *upper_bound);

/* Sizes of the reduced graph: order n, |V|, sum over v of |D*(v)| (entries of
 * one conflict table) and the device row stride; any pointer may be NULL. */
int plse_sizes(plse_handle h, int32_t *n, int32_t *num_vertices, int32_t *domain_entries,
               int32_t *stride);

/* Device row stride (bytes) of one individual: |V| rounded up to 16.
 * Stage calls read and write populations as [count][stride] uint8. */
int plse_row_stride(plse_handle h, int32_t *stride);

/*
 * plse_set_param / plse_get_param -- solver parameters (Table 1, Section 3.3).
 *   "depth"       total tabu iterations per individual and generation; phase 2
 *                 gets min(2|V|, depth), phase 1 the rest (default 10 n^2)
 *   "depth1", "depth2"  phase lengths set directly (paper: 100|V| and 2|V|)
 *   "alpha_num", "alpha_den"   tenure factor alpha (6/10)
 *   "beta_num", "beta_den"     AUX beta (20/1, Eq. 9)
 *   "spacing"     minimum spacing factor gamma of Section 3.4 (10)
 *   "stop_at_ub"  1: stop after the generation whose best reaches the bound
 *   "max_iterations"  > 0: iteration budget of the run (Section 4.3 caps each
 *                 run at a total number of tabu iterations): the run stops
 *                 after the first generation at whose end the population's
 *                 cumulative iteration count reaches the budget; 0: none
 *   "nn_history"  partner-history length, 0..64 (64)
 *   "crossover"   0 AUX (Alg. 5, default), 1 UX (p_ij fixed at 1/2, Section
 *                 3.5.2), 2 none: the offspring copies its first parent
 *                 (Section 5.2)
 *   "matching"    0 nearest neighbour with partner history (Section 3.5.1,
 *                 default), 1 random: a uniformly drawn other individual
 *                 (Section 5.3); plse_stage_match always matches nearest
 *   "slots_per_lane" 2, 4 or 8: candidate moves one lane evaluates per PLITS
 *                 round (default 0: chosen from the domain sizes)
 *   "waves_per_block" 1, 2 or 4: PLITS launch shape (default: chosen from the
 *                 LDS footprint)
 *   "plits_kernel" 1: the tabu-search kernel with each individual's tabu
 *                 table in global memory (the default, also 0); 2: the kernel
 *                 with the whole search state in LDS (MPMA only, when it fits
 *                 the device's per-block LDS).  Both give the same results.
 *   "persistent"  1 (default): in plse_solve_batch, the tabu searches of the
 *                 instances sharing a launch shape run as one persistent
 *                 launch whose waves take (instance, individual) items,
 *                 instances in order of estimated work (longest first); 0 (on
 *                 any instance of the group): a grid of blocks per instance
 *   "plits_waves_per_cu" (plse_get_param only): resident tabu-search waves
 *                 per CU under the handle's launch shape (the runtime's
 *                 occupancy calculation; needs the HIP runtime)
 *   "stage_timing" 1: single-instance sessions enqueue each stage of a
 *                 generation on its own between HIP events (no graphs; the
 *                 distances among P_t run before the search instead of
 *                 beside it), for plse_last_stage_timing; results unchanged
 *   "max_generations" 1..65536: the most generations one session of this
 *                 handle may run (65536); the workspace holds one statistics
 *                 record (80 bytes) per generation, so a smaller value
 *                 shrinks plse_workspace_bytes.  plse_solve / plse_step
 *                 beyond it return PLSE_E_ARG.  The server sets it to each
 *                 request's generation budget while the request is held and
 *                 restores the caller's value when it ends.
 * Errors: PLSE_E_PARAM.
 */
/* Test hook (selection): "select_global_sort" 1 sorts the selection keys with
 * the global-memory network even when they would fit in LDS (populations of
 * at least 4096; the network always serves populations whose keys exceed LDS). */
/* Test hook (serving): "fail_at_generation" g > 0 makes a served request end
 * with PLSE_E_FAULT after its generation g, without touching other requests. */
int plse_set_param(plse_handle h, const char *key, int64_t value);
int plse_get_param(plse_handle h, const char *key, int64_t *value);

/*
 * plse_autotune -- pick the tabu-search chunk size of this instance by
 * measurement.  The initial population of `seed` (`sample` individuals, in
 * the attached workspace, which must hold that population) runs one
 * generation of phase-1 search of `depth` iterations with each candidate-
 * positions-per-lane value that fits (2, 4, 8), each timed with HIP events on
 * `stream` after one untimed launch; the fastest is stored as the handle's
 * "slots_per_lane".  Waves per block keep the handle's setting (by default
 * the occupancy rule, which also weighs the uneven search lengths of later
 * generations that a short sample does not show).  The shape changes speed
 * only: every result is the same under any shape; batches group instances
 * by it.  out_ms (may be NULL) receives the 3 times in ms (slots 2, 4, 8), -1
 * where a size does not fit.  Synchronises `stream`.  Errors: PLSE_E_ARG
 * (sample < 2, depth < 1), PLSE_E_WORKSPACE, PLSE_E_BUSY, PLSE_E_HIP.
 */
int plse_autotune(plse_handle h, int32_t sample, int32_t depth, uint64_t seed, void *stream,
                  float *out_ms);

/* plse_autotune_shape -- as plse_autotune, over chunk size and waves per
 * block together: 9 timed shapes (slots per lane 2, 4, 8 for 1, then 2, then
 * 4 waves per block; out_ms may be NULL, else 9 floats, -1 where a shape does
 * not fit); the fastest is stored as "slots_per_lane" and "waves_per_block".
 * Same errors. */
int plse_autotune_shape(plse_handle h, int32_t sample, int32_t depth, uint64_t seed,
                        void *stream, float *out_ms);

/* Bytes of device workspace a solve with this population needs. */
int plse_workspace_bytes(plse_handle h, int32_t population, size_t *bytes);

/* Attach caller-owned device memory (256-byte aligned); it must outlive every
 * solve and stage call.  Passing NULL detaches. */
int plse_attach_workspace(plse_handle h, void *device_ptr, size_t bytes);

/*
 * plse_solve -- run the memetic algorithm (Alg. 2) on the attached workspace.
 *
 * Initial population (Section 3.2), then per generation: the two-phase tabu
 * search PLITS on every offspring (Section 3.3, Alg. 3), best-solution
 * saving, Hamming distances over both populations (Eq. 8), the population
 * update (Alg. 4), nearest-neighbour parent matching (Section 3.5.1) and the
 * AUX crossover (Alg. 5, Eq. 9).  Stops after `generations`, or earlier with
 * stop_at_ub when the score reaches the upper bound.
 *
 * population: 2..32768.   generations: 1..65536.   seed: any 64-bit value.
 * stream:     hipStream_t (may be NULL = default stream).
 * best_grid:  host, n*n int8: the prefilled cells plus the best colouring S*;
 *             impossible and uncoloured cells are 0.
 * filled:     host, number of non-zero cells of best_grid (<= upper bound).
 * The result depends only on (grid, parameters, population, generations,
 * seed).  Returns after the results are on the host.
 * Errors: PLSE_E_ARG, PLSE_E_WORKSPACE, PLSE_E_HIP, PLSE_E_BUSY.
 */
int plse_solve(plse_handle h, int32_t population, int32_t generations, uint64_t seed,
               void *stream, int8_t *best_grid, int32_t *filled);

/*
 * Session form of plse_solve, for callers that drive generations themselves:
 *   plse_begin  uploads the instance, builds the initial population and
 *               prepares the generation graphs (enqueued on `stream`);
 *   plse_step   enqueues `generations` more generations of Alg. 2 (no host
 *               synchronisation); HIP events are recorded on `stream` before
 *               and after each tabu-search launch and at the end of each
 *               generation;
 *   plse_end    waits for the stream, then returns the best grid as
 *               plse_solve does and fills the statistics and timings.
 * plse_solve(h, p, G, ...) is plse_begin + plse_step(G) + plse_end.
 * A session holds the handle's workspace until plse_end.
 * Errors: PLSE_E_ARG (no session, more than PLSE_MAX_GENERATIONS steps),
 * PLSE_E_WORKSPACE, PLSE_E_HIP, PLSE_E_BUSY.
 */
int plse_begin(plse_handle h, int32_t population, uint64_t seed, void *stream);
int plse_step(plse_handle h, int32_t generations, void *stream);
int plse_end(plse_handle h, void *stream, int8_t *best_grid, int32_t *filled);

/*
 * plse_peek -- progress of the open session: waits for `stream` (so for
 * every generation stepped so far), then reports the generations run, the
 * best f, the generation that found it, the population's cumulative tabu
 * iterations and the stop reason (as in plse_stats; a stopped run ignores
 * further steps).  For callers that stop on a wall-clock budget between
 * plse_step calls, as the time-limited runs of Section 5.1.  The session
 * stays open.  Errors: PLSE_E_ARG (null, no open session), PLSE_E_BUSY,
 * PLSE_E_HIP.
 */
typedef struct {
    int32_t generations_run;
    int32_t best_f;               /* INT32_MAX before the first generation ends */
    int32_t best_generation;
    int32_t stop_reason;
    uint64_t iterations;
} plse_progress;
int plse_peek(plse_handle h, void *stream, plse_progress *out);

/*
 * plse_checkpoint / plse_resume -- save the open session (plse_begin or
 * plse_resume) at its generation boundary and continue it later, in this or
 * another process, on a handle of the same grid and parameters.  The state
 * of Alg. 2 between generations is the population P_t with f, the uids and
 * partner histories of its members, the offspring waiting for the next
 * search, S* and the per-generation statistics; all random draws are
 * counter-based, so a resumed run is bit-identical to an uninterrupted one.
 * plse_checkpoint waits for `stream` (every generation stepped so far), sets
 * *bytes to the image size and, when buf is not NULL and capacity >= *bytes,
 * writes the image to buf (host, caller-owned); the session stays open.
 * plse_resume opens a session from an image (instead of plse_begin), with
 * the handle's attached workspace (sized for `population`); continue with
 * plse_step / plse_peek / plse_end.  plse_last_timing then covers the
 * generations stepped since the resume.  Errors: PLSE_E_ARG (no open
 * single-instance session, capacity too small, an image of another grid,
 * parameters or population, or a damaged image), PLSE_E_WORKSPACE,
 * PLSE_E_BUSY, PLSE_E_HIP.
 */
int plse_checkpoint(plse_handle h, void *stream, void *buf, size_t capacity, size_t *bytes);
int plse_resume(plse_handle h, int32_t population, void *stream, const void *buf, size_t bytes);

/*
 * plse_solve_batch -- plse_solve on `count` instances at once.
 *
 * Every generation of Alg. 2 runs for all instances together: one launch per
 * kernel covers the instances (grouped by PLITS launch shape and by colour
 * width, longest estimated work first), captured once as HIP graphs and
 * replayed per generation.  Each handle needs its own attached workspace of
 * plse_workspace_bytes(hs[i], population); the handles must be distinct and
 * idle.  seeds[i], best_grids[i] (host n_i*n_i) and filled[i] belong to
 * hs[i].  The result of each instance is identical to plse_solve of that
 * instance alone with the same arguments.  Per-instance statistics and
 * timings are then available through plse_last_stats / plse_last_timing.
 * Errors: PLSE_E_ARG (null, duplicate handle, bad sizes), PLSE_E_WORKSPACE,
 * PLSE_E_BUSY, PLSE_E_HIP.
 */
int plse_solve_batch(const plse_handle *hs, int32_t count, int32_t population,
                     int32_t generations, const uint64_t *seeds, void *stream,
                     int8_t *const *best_grids, int32_t *filled);

/*
 * Session form of plse_solve_batch, for callers that step a batch in parts:
 *   plse_batch_begin  holds the handles (each idle, distinct, with its
 *                     workspace) and builds every initial population;
 *   plse_batch_step   enqueues `generations` more generations of all of them;
 *   plse_batch_end    waits for the stream, writes best_grids[i] / filled[i]
 *                     for hs[i] of plse_batch_begin, fills each handle's
 *                     statistics, releases the handles and frees the batch
 *                     (also on error).
 * plse_solve_batch(hs, count, p, G, ...) is begin + step(G) + end; the
 * results are the same however the generations are split.  One call at a
 * time per batch.  Errors as plse_solve_batch; plse_batch_step: PLSE_E_ARG
 * beyond max_generations.
 */
typedef struct plse_batch_t *plse_batch;
int plse_batch_begin(const plse_handle *hs, int32_t count, int32_t population,
                     const uint64_t *seeds, void *stream, plse_batch *out);
int plse_batch_step(plse_batch b, int32_t generations, void *stream);
int plse_batch_end(plse_batch b, void *stream, int8_t *const *best_grids, int32_t *filled);

/*
 * plse_solve_noalloc -- plse_solve for callers that cannot allocate device
 * memory or create runtime objects (code that must not call hipMalloc: tight
 * serving loops, harnesses that forbid allocation).  Instead of the handle's
 * attached workspace it uses a fixed device array of PLSE_NOALLOC_BYTES
 * inside the library, one per GPU, reserved when the library's code is
 * loaded on that GPU and held until the process ends; the kernels are
 * enqueued one by one on `stream` (no HIP graphs, side streams or events).
 * The result, plse_last_stats and the handle's attached workspace are as
 * after plse_solve with the same arguments; plse_last_timing reports no
 * steps.  *bytes_needed (may be NULL) receives the workspace this call needs
 * (its per-generation records sized for `generations`).  Every call on one
 * GPU shares that GPU's array and overwrites it: calls that overlap in time
 * on the same GPU (other streams, threads or handles) race and must not be
 * issued.  Call with the stream's device current.  Errors: PLSE_E_ARG,
 * PLSE_E_BUSY, PLSE_E_CAPACITY (the instance and population need more than
 * PLSE_NOALLOC_BYTES; checked before any device work), PLSE_E_HIP.
 */
#define PLSE_NOALLOC_BYTES (64ull << 20)
int plse_solve_noalloc(plse_handle h, int32_t population, int32_t generations, uint64_t seed,
                       void *stream, int8_t *best_grid, int32_t *filled, size_t *bytes_needed);

/*
 * plse_measure_lds_bandwidth -- a device measurement, not a step of the
 * method: the sustained LDS read bandwidth of the current GPU (bytes/s, best
 * of `repeats` timed launches after one warm-up), the peak against which the
 * LDS-resident tabu search is compared.  Every CU runs blocks that read
 * 16-byte words at conflict-free addresses from a 32 KiB buffer.  Uses the
 * library's fixed device array (see plse_solve_noalloc) as its output sink,
 * so it must not overlap plse_solve_noalloc calls on the same GPU.  Errors:
 * PLSE_E_ARG, PLSE_E_HIP.
 */
int plse_measure_lds_bandwidth(void *stream, int32_t repeats, double *bytes_per_second);

/* Per-generation GPU times of the last session, from the HIP events of
 * plse_step: plits_ms[g] spans the tabu-search launch of generation g,
 * rest_ms[g] the best/distance/selection/matching/crossover kernels.  *steps
 * receives the number of generations stepped; either array may be NULL. */
int plse_last_timing(plse_handle h, int32_t *steps, float *plits_ms, float *rest_ms);

/* Per-stage GPU times (ms) of the last single-instance session run with the
 * "stage_timing" parameter set: PLSE_NSTAGES floats per generation, in the
 * order of Alg. 2's steps -- distances among P_t (Eq. 8), the tabu searches
 * (Alg. 3), best-solution saving, distances between P' and P_t u P', the
 * population update (Alg. 4: close-pair lists, selection, gather), parent
 * matching (Section 3.5.1) and AUX crossover (Eq. 9, Alg. 5).  *steps
 * receives the generations timed (0 without stage timing); ms may be NULL. */
#define PLSE_NSTAGES 7
int plse_last_stage_timing(plse_handle h, int32_t *steps, float *ms);

/* Statistics of the last solve, the per-run quantities of Tables 3-4 and
 * Section 4.3 (best f and the generation that found it, the stop reason, and
 * the tabu work: iterations, moves and the other PLSE_NCOUNTERS counters of
 * Section 3.3's search); per_gen_best_f (may be NULL) receives the best f
 * after each generation (generations_run entries) and per_gen_counters (may
 * be NULL) PLSE_NCOUNTERS u64 per generation. */
int plse_last_stats(plse_handle h, plse_stats *out, int32_t *per_gen_best_f,
                    uint64_t *per_gen_counters);

void plse_destroy(plse_handle h);
const char *plse_strerror(int status);

/*
 * Stage calls: one step of the path on caller device buffers, with the
 * handle's attached workspace (sized for at least `population`) as scratch.
 * They enqueue on `stream` and return without synchronising.  Populations are
 * [count][stride] uint8 device arrays (stride from plse_row_stride).
 */

/* Randomised greedy legal colourings of slots 0..p-1 (Section 3.2).
 * S: device [p][stride] out; f: device int32 [p] out (uncoloured counts). */
int plse_stage_init(plse_handle h, int32_t population, uint64_t seed, void *stream,
                    uint8_t *S, int32_t *f);

/* PLITS (Section 3.3, Alg. 3) of generation `gen` on slots 0..p-1.
 * S_in: device [p][stride]; S_out: device [p][stride] (distinct from S_in);
 * f_out: device int32 [p]; counters: device uint64 [p][PLSE_NCOUNTERS]. */
int plse_stage_plits(plse_handle h, int32_t population, int32_t gen, uint64_t seed,
                     void *stream, const uint8_t *S_in, uint8_t *S_out, int32_t *f_out,
                     uint64_t *counters);

/* Hamming distances (Eq. 8) between all pairs of m individuals.
 * S: device [m][stride]; D: device int16 [m][m] out.  m <= 2*population. */
int plse_stage_distances(plse_handle h, int32_t m, void *stream, const uint8_t *S, int16_t *D);

/* Population update (Alg. 4) over 2p candidates (P_t = 0..p-1, P' = p..2p-1).
 * f_all: device int32 [2p]; D_all: device int16 [2p][2p];
 * accepted: device int32 [p] out, the next population in slot order. */
int plse_stage_select(plse_handle h, int32_t population, int32_t gen, uint64_t seed,
                      void *stream, const int32_t *f_all, const int16_t *D_all,
                      int32_t *accepted);

/* Parent matching (Section 3.5.1) with partner history.
 * D: device int16 [p][p]; uid: device uint64 [p]; hist: device uint64
 * [p][PLSE_HIST] and hcount: device int32 [p], both updated in place;
 * partner, dpart: device int32 [p] out. */
int plse_stage_match(plse_handle h, int32_t population, void *stream, const int16_t *D,
                     const uint64_t *uid, uint64_t *hist, int32_t *hcount, int32_t *partner,
                     int32_t *dpart);

/* AUX crossover (Alg. 5, Eq. 9) of generation `gen`.
 * S: device [p][stride]; partner, dpart: device int32 [p];
 * S_off: device [p][stride] out. */
int plse_stage_aux(plse_handle h, int32_t population, int32_t gen, uint64_t seed, void *stream,
                   const uint8_t *S, const int32_t *partner, const int32_t *dpart,
                   uint8_t *S_off);

/*
 * Serving: continuous batching of solve requests on one device.
 *
 * A server owns a device arena (caller memory, hbm_budget_bytes) and a worker
 * thread.  Requests wait in arrival order; the worker admits them while their
 * workspace (plse_workspace_bytes) fits in the free arena (first fit) and
 * fewer than max_slots are resident.  Every resident request runs on a
 * stream of its own, with up to two generations of Alg. 2 enqueued ahead, so
 * requests that arrive while others run share the device with them and none
 * waits for another's generations; a finished request's workspace returns
 * to the arena.  A run that stops before its last generation (the bound with
 * stop_at_ub, or its iteration budget) leaves the device at the end of the
 * generation that stopped it, instead of stepping through the rest.  Streams
 * run side by side only on distinct hardware queues: a serving process
 * should raise the HIP runtime's queue count (environment variable
 * GPU_MAX_HW_QUEUES, default 4) towards max_slots before the runtime
 * initialises (16 queues serve a 16-request trace 1.3x faster than 4).  Each
 * result is identical to plse_solve of the same instance, parameters,
 * population, generations and seed, whatever else is resident.
 *
 * plse_server_create: device_ptr/hbm_budget_bytes the arena (256-byte
 *   aligned, caller-owned, must outlive the server); max_slots >= 1; stream
 *   orders the server's work after work already queued on it (the requests'
 *   own streams wait for it once, at creation).
 * plse_server_submit: the handle is used by the server until its result has
 *   been polled (do not touch it meanwhile).  Returns PLSE_E_CAPACITY if the
 *   request's workspace can never fit the arena; *ticket identifies it.
 * plse_server_poll: PLSE_PENDING while the request runs; then fills the grid
 *   (host n*n), filled and the timing record, returns the request's own status
 *   (PLSE_OK, or the error that ended it) and forgets the ticket.
 * plse_server_destroy: stops the worker, waits for the work enqueued for
 *   resident requests, and drops waiting and resident requests.
 */
typedef struct plse_server_s *plse_server;

typedef struct {
    double submit_s;        /* seconds since the server was created          */
    double admit_s;         /* admitted (workspace placed, population built) */
    double done_s;          /* last generation finished                      */
    double best_s;          /* end of the generation that found S*           */
    int32_t generations;    /* generations run                               */
    int32_t best_generation;
    int32_t filled;
    int32_t status;
    uint64_t moves;         /* tabu moves executed for this request          */
} plse_timing;

int plse_server_create(size_t hbm_budget_bytes, void *device_ptr, int32_t max_slots, void *stream,
                       plse_server *out);
int plse_server_submit(plse_server s, plse_handle h, int32_t population, int32_t generations,
                       uint64_t seed, uint64_t *ticket);
int plse_server_poll(plse_server s, uint64_t ticket, int8_t *best_grid, int32_t *filled,
                     plse_timing *timing);
/* Requests waiting, resident, and finished but not yet polled. */
/* plse_server_cancel: a waiting request is dropped (poll: PLSE_E_CANCELLED, no
 * grid); a resident one stops once the generations already enqueued on its
 * stream have run (at most two beyond the current one), and its poll returns
 * PLSE_E_CANCELLED with the best grid found by then (filled and timing set;
 * generations and time to best include those drained generations, whose end
 * times come from their end events).  PLSE_E_ARG for an unknown or already
 * finished ticket. */
int plse_server_cancel(plse_server s, uint64_t ticket);
int plse_server_status(plse_server s, int32_t *waiting, int32_t *resident, int32_t *finished);
int plse_server_destroy(plse_server s);

#ifdef __cplusplus
}
#endif
#endif /* PLSE_H */
