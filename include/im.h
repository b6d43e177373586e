/*
 * im.h -- C ABI of the MI355X sketch-based influence-maximisation library
 * (libimx.so).  The method is DiFuseR's (Gokturk and Kaya): Monte-Carlo
 * independent-cascade simulations whose live edges are decided by hashing
 * (Section 2.2, Eq. 1-2), one count-distinct register per (vertex,
 * simulation) (Section 2.3, Eq. 3-5; Section 3.1), pull-based register
 * propagation (Section 3.2, Alg. 2), harmonic-mean cardinality estimates
 * (Section 3.1, Eq. 7), greedy selection with a union-frontier covering
 * cascade (Section 3.3, Alg. 3) and the error-adaptive rebuild test
 * (Section 4, Alg. 4).  All computation runs in HIP kernels on one gfx950 GPU.
 *
 * Conventions for every entry point:
 *   - Pointers named *_host are host memory owned by the caller; the library
 *     copies inputs and writes outputs, and keeps no reference after return.
 *   - Handles are owned by the library until the matching *_free call.  A graph
 *     must outlive every sketch built on it.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a handle is ordered on the stream it was created with;
 *     functions that return host results synchronise that stream.
 *   - Errors: a status code is returned and a message is kept per thread
 *     (im_last_error).  Nothing throws across the ABI.  A failed call leaves
 *     existing handles unchanged; *out is left NULL.
 *   - One thread at a time per handle; distinct handles are independent.
 */
#ifndef IMX_IM_H
#define IMX_IM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum im_status {
    IM_OK = 0,
    IM_EINVAL = 1,  /* malformed argument (CSR, probability, J, K ...)        */
    IM_ENOMEM = 2,  /* device memory (or an admission budget) too small       */
    IM_EDEVICE = 3, /* HIP runtime error or no gfx950 device                  */
    IM_ESTATE = 4   /* call not allowed in the handle's current state         */
} im_status;

typedef struct im_graph im_graph;
typedef struct im_sketch im_sketch;

/* Counters of one sketch.  Times are device time measured with HIP events on
 * the sketch's stream. */
typedef struct im_stats {
    int32_t build_sweeps;    /* propagation sweeps of the initial build, including
                                the final sweep that changed nothing            */
    int32_t rebuilds;        /* rebuilds triggered by the error-adaptive test   */
    int64_t total_sweeps;    /* sweeps over the initial build and all rebuilds  */
    int64_t cascade_levels;  /* union-frontier levels over all cascades         */
    double build_ms;         /* im_sketch_build: fill + propagation + estimate  */
    double select_ms;        /* im_select_seeds, end to end                     */
    double propagate_ms;     /* device time of the steps that ran this query's
                                propagation sweeps (shared steps count fully;
                                profiling level >= 1, else 0)                   */
    double cascade_ms;       /* device time of the steps that ran this query's
                                covering cascades (shared steps count fully;
                                profiling level >= 1, else 0)                   */
    int64_t prop_launches;   /* propagation kernel launches; a step launches a
                                fixed number of sweeps, and those after the
                                build converged return at once                  */
    double prop_kernel_ms;   /* sum of per-launch propagation kernel times
                                (profiling level >= 1, else 0)                  */
    /* Algorithmic traffic of the propagation sweeps, counted by the kernel's
     * instrumented variant when profiling level 2 is on (else all 0):
     *   bytes = (8 + J)*rows_visited + J*rows_changed + 8*arcs_active + 64*sectors
     * summed over sweeps, where rows_visited = rows with at least one arc whose
     * head changed in the previous sweep (row bounds and own registers read),
     * rows_changed = rows stored, arcs_active = such arcs (head id and
     * threshold), sectors = 64-byte sectors of their heads' rows that hold
     * simulations where the arc is live.  The other counters are the kernel's
     * own events: tasks visited, rows staged with candidates, changed 32-bit
     * words x 4 stored, arcs whose head id was read. */
    double prop_alg_bytes;
    int64_t prop_tasks, prop_rows_read, prop_bytes_written;
    int64_t prop_arcs_scanned, prop_arcs_active, prop_sectors;
    int64_t prop_rows_visited, prop_rows_changed;
} im_stats;

/* Message of the last failed call on this thread ("" if none). */
const char* im_last_error(void);

/* Library version (major, minor). */
im_status im_version(int32_t* major, int32_t* minor);

/*
 * Device memory hooks, so that a host framework (for example PyTorch's caching
 * allocator) owns the device memory of the library (the problem statement's
 * inputs and the method's state are otherwise allocated with hipMalloc).
 *   alloc(bytes, ctx)  returns a device pointer aligned to at least 16 bytes,
 *                      or NULL when it cannot (the calling im_* function then
 *                      fails with IM_ENOMEM and changes nothing);
 *   free_(ptr, ctx)    returns a pointer alloc gave.
 * Process-wide; applies to graphs, sketches and engines created afterwards.
 * Every buffer is returned to the hooks that allocated it, also after the
 * hooks change.  Both NULL restores hipMalloc / hipFree.  Errors: IM_EINVAL
 * when exactly one of the two is NULL.  The hooks may be called from any
 * thread that calls into the library.
 */
typedef void* (*im_alloc_fn)(size_t bytes, void* ctx);
typedef void (*im_free_fn)(void* ptr, void* ctx);
im_status im_set_allocator(im_alloc_fn alloc, im_free_fn free_, void* ctx);

/*
 * Process-wide measurement switch for engine steps issued afterwards:
 *   0  no device timing (the default; propagate_ms, cascade_ms and
 *      prop_kernel_ms in im_stats stay 0),
 *   1  per-launch propagation kernel times and per-phase device times (HIP
 *      events around the launches; not in HIP-graph mode),
 *   2  as 1, and the instrumented propagation kernel runs, counting the
 *      algorithmic traffic reported in im_stats (slower; for roofline
 *      reports, never for timing).
 * Results are identical at every level.  Errors: IM_EINVAL for other levels.
 */
im_status im_set_profiling(int32_t level);

/*
 * Load a directed graph G=(V,E) with IC edge probabilities w (Section 2.1;
 * problem input of Alg. 4).
 *   n       number of vertices, 1 <= n < 2^31.
 *   m       number of arcs, 0 <= m < 2^40.
 *   rowptr_host  int64[n+1], CSR by source: out-arcs of u are
 *           col_host[rowptr[u] .. rowptr[u+1]).  rowptr[0]=0, non-decreasing,
 *           rowptr[n]=m.
 *   col_host     int32[m] destination ids in [0,n), strictly increasing within
 *           each row (parallel arcs must be merged by the caller into one arc
 *           with the compound probability, as Section 2.1 describes).
 *   p_host       float32[m] probability of each arc in [0,1] (no NaN).  It is
 *           turned on the device into the 31-bit fixed-point threshold
 *           W = min(2^31, floor(p * 2^31)) used by the live test of Eq. 2.
 *   stream  stream for the upload and all later work on the graph.
 *   out     receives the handle.
 * Errors: IM_EINVAL for any violation above (message names the first bad
 * index), IM_ENOMEM if the device cannot hold the graph, IM_EDEVICE.
 */
im_status im_graph_load(int64_t n, int64_t m, const int64_t* rowptr_host, const int32_t* col_host,
                        const float* p_host, void* stream, im_graph** out);

/* Number of vertices and arcs of a loaded graph. */
im_status im_graph_info(const im_graph* g, int64_t* n, int64_t* m);

void im_graph_free(im_graph* g);

/*
 * Build the sketches of all vertices (Alg. 4 before its greedy loop):
 * J simulations with random values X drawn from `seed` and sorted
 * (Section 4.1), registers filled with each vertex's own rank (Alg. 1,
 * Eq. 3) and propagated backwards along live arcs until no register
 * changes (Alg. 2, Eq. 5).  Then per-vertex estimate terms are computed.
 *   J     registers (= simulations) per vertex: a multiple of 64 in [64, 4096].
 *   seed  64-bit seed of the simulation values and of the register hashes.
 * The register array takes n*J bytes of device memory, vertex-major with each
 * row's registers in increasing simulation order (Section 3.1).
 * Errors: IM_EINVAL (bad J, NULL graph), IM_ENOMEM, IM_EDEVICE.
 */
im_status im_sketch_build(const im_graph* g, int32_t J, uint64_t seed, void* stream, im_sketch** out);

/*
 * Greedy selection of K seeds (Alg. 4 loop): per pick, harmonic-mean
 * estimates (Eq. 7) -> argmax over non-seeds (exact rational compare of
 * J_u^2/H_u, lowest id on ties) -> covering cascade from the pick (Alg. 3) ->
 * score T (covered (vertex, simulation) pairs) -> if the pick is not the
 * last and 100*(T - T_old) > T, refill uncovered registers and propagate
 * again, then T_old = T.
 *   K          1 <= K <= n.
 *   seeds_host int32[K] output, in pick order.
 *   spread_out optional double: T_K / J, the expected spread of the seed set
 *              over the J simulations.
 *   est_host   optional double[K]: estimated marginal gain of each pick,
 *              alpha_J * 2^33 * J_s^2 / (J * H_s) (0 when J_s = 0).
 *   T_host     optional uint64[K]: T after each pick's cascade.
 *   stats_out  optional counters and device times.
 * The sketch is consumed: a second call returns IM_ESTATE.
 * Errors: IM_EINVAL (K out of range, NULL seeds), IM_ESTATE, IM_EDEVICE.
 */
im_status im_select_seeds(im_sketch* s, int32_t K, int32_t* seeds_host, double* spread_out, double* est_host,
                          uint64_t* T_host, im_stats* stats_out);

/*
 * Parity hook: run the greedy loop of im_select_seeds(s, K, ...) only up to
 * pick number k_stop (0-based) and pause before it, so a test can compare the
 * state every pick reads (Alg. 4 loop: estimate terms, registers after each
 * rebuild, covered registers) with a reference.  At the pause the registers
 * (im_sketch_registers / im_sketch_register_rows) are those pick k_stop
 * reads, after every cascade so far and any rebuild, and the estimate terms
 * (im_sketch_estimates) are current.  A later call with a larger k_stop goes
 * on; im_select_seeds(s, K, ...) with the same K finishes the loop and
 * returns every output as if it had run uninterrupted (results never depend
 * on pauses).
 *   K           as for im_select_seeds; the same K on every call of one sketch.
 *   k_stop      picks to make before pausing, in [0, K) and not below the
 *               picks already made.
 *   seeds_host  optional int32[k_stop]: the picks made so far.
 *   T_host      optional uint64[k_stop]: T after each of their cascades.
 * Errors: IM_EINVAL (K or k_stop out of range, K differing from the paused
 * selection's), IM_ESTATE (selection finished), IM_EDEVICE.
 */
im_status im_select_seeds_until(im_sketch* s, int32_t K, int32_t k_stop, int32_t* seeds_host, uint64_t* T_host);

/* Copy the current registers to host memory uint8[n*J] (vertex-major; covered
 * registers read 0, uncovered ones hold rank values 1..33).  Parity hook. */
im_status im_sketch_registers(const im_sketch* s, uint8_t* regs_host);

/* Copy selected register rows to host memory: rows_host int32[nrows] vertex ids
 * in [0, n), regs_host uint8[nrows*J] receives the rows in that order.  Parity
 * hook for sketches too large to download whole.  Errors: IM_EINVAL for a bad
 * id or NULL pointer. */
im_status im_sketch_register_rows(const im_sketch* s, const int32_t* rows_host, int32_t nrows, uint8_t* regs_host);

/* Copy the current per-vertex estimate terms: Ju_host uint32[n] = number of
 * uncovered registers, Hu_host uint64[n] = sum over them of 2^(33 - M).  Either
 * pointer may be NULL.  Parity hook. */
im_status im_sketch_estimates(const im_sketch* s, uint32_t* Ju_host, uint64_t* Hu_host);

/* Counters of the sketch so far. */
im_status im_sketch_stats(const im_sketch* s, im_stats* out);

/* Sorted simulation values X (uint32[J], 31-bit) of the sketch.  Parity hook. */
im_status im_sketch_sim_values(const im_sketch* s, uint32_t* X_host);

void im_sketch_free(im_sketch* s);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the query of
 * im_sketch_build(g, J, seed) followed by im_select_seeds(K), with the same
 * kernels and bit-identical results, but without allocating any device or
 * pinned host memory.  Its working buffers live in a fixed device array of
 * 64 MiB that the library holds per device for the life of the process; the
 * registers live in a buffer the caller passes.
 *   g             graph on the current device.
 *   J, seed, K    as for im_sketch_build and im_select_seeds.
 *   registers_dev device buffer of n*J bytes (uint8, vertex-major), owned by
 *                 the caller; its contents on entry are ignored, and on return
 *                 it holds the final registers (covered registers 0), as
 *                 im_sketch_registers would after im_select_seeds.
 *   seeds_host    int32[K] output, in pick order.
 *   spread_out    optional double: T_K / J.
 *   est_host      optional double[K]: estimate of each pick.
 *   stream        stream of the call's work (NULL = null stream); the call
 *                 returns after the work has finished.
 * Working memory needed: about 24 bytes per vertex, 16 per out-task and 4 per
 * in-task (a graph of a million vertices fits); a query that needs more than
 * 64 MiB returns IM_EINVAL and does nothing.  Every call on one device shares
 * that device's array and overwrites it: calls that overlap on one device
 * (from several threads, or on several streams) race and must be serialised.
 * Errors: IM_EINVAL (NULL pointer, bad J or K, working memory above the
 * maximum), IM_EDEVICE.
 */
im_status im_select_seeds_noalloc(const im_graph* g, int32_t J, uint64_t seed, int32_t K, uint8_t* registers_dev,
                                  int32_t* seeds_host, double* spread_out, double* est_host, void* stream);

/*
 * Engines run many queries (graph, J, seed, K) together: every query follows
 * exactly the steps of im_sketch_build + im_select_seeds, and the engine
 * advances all of them one stage per im_engine_step, sharing kernel launches
 * (one batched launch per kernel kind) and one host synchronisation per step.
 * A query's results do not depend on the other queries in the engine.
 * Queries may be submitted at any time (continuous admission); a submission
 * that would exceed the engine's device-memory budget returns IM_ENOMEM and
 * changes nothing, so the caller can retry after results are collected.
 *
 *   max_queries       concurrent queries (slots), 1..4096.
 *   hbm_budget_bytes  device memory the engine's queries may hold (0: the
 *                     device's free memory at creation).
 *   stream            stream of all the engine's work.
 * Graphs must outlive the engine's queries on them.
 */
typedef struct im_engine im_engine;

im_status im_engine_create(int32_t max_queries, uint64_t hbm_budget_bytes, void* stream, im_engine** out);

/* Scheduling parameters of an engine (they change speed, never results):
 *   group_first, group_rest  lanes per propagation task (16, 32 or 64) in the
 *                            first sweep after a fill and in later sweeps, or
 *                            0 for the packed kernel (each wave takes
 *                            max(1, min(16, B / J)) tasks at once, B = 2048
 *                            bytes, or 1024 / 4096 from the environment
 *                            variable IMX_PACK_BYTES, read once per process);
 *   rounds_per_step          sweeps / cascade levels launched per step (1..16);
 *   dense_div                a sweep visits every task instead of an active
 *                            list when more than n / dense_div rows changed in
 *                            the previous sweep (>= 1);
 *   use_graphs               1: every step launches every kernel kind for
 *                            every running query (records of queries in
 *                            other stages are inactive), so the launch
 *                            sequence changes only when a query is admitted
 *                            or finishes; it is captured in a HIP graph the
 *                            first time it occurs and replayed while it
 *                            repeats (no per-launch kernel times then); it
 *                            is meant for many queries in one engine (with
 *                            one large query it was measured 46% slower);
 *                            0: direct launches of the queries in each stage;
 *   grid_cap                 at most this many workgroups in any launch of
 *                            the engine (0: no cap), e.g. to keep an engine of
 *                            small queries from crowding out another engine's
 *                            large ones on a shared device;
 *   tails                    single-workgroup tail kernels for small
 *                            frontiers (many sweeps or cascade levels in one
 *                            launch): 0 off, 1 on, 2 only for graphs whose
 *                            largest in- and out-degree is at most 64.
 * Defaults: 0, 0, 8, 16, 0, 0, 2; the environment variables IMX_GROUP_FIRST,
 * IMX_GROUP, IMX_ROUNDS, IMX_DENSE_DIV, IMX_GRAPHS and IMX_TAIL override them at
 * engine creation (an out-of-range value makes creation fail with IM_EINVAL).
 * IMX_PROP_GRID (>= 1), read at engine creation, caps the workgroups of a
 * propagation launch (a test of schedule independence; never faster).
 * A launch that carries several queries (and every launch in graph mode)
 * divides its workgroups among them on the device, by each query's current
 * work; IMX_DYN_SPLIT=0 at engine creation divides them on the host by graph
 * size instead. */
typedef struct im_tuning {
    int32_t group_first;
    int32_t group_rest;
    int32_t rounds_per_step;
    int32_t dense_div;
    int32_t use_graphs;
    int32_t grid_cap;
    int32_t tails;
} im_tuning;

im_status im_engine_set_tuning(im_engine* e, const im_tuning* t);
im_status im_engine_get_tuning(const im_engine* e, im_tuning* t);

/* Steps taken, graphs captured and graph replays of an engine (diagnostics). */
im_status im_engine_counters(const im_engine* e, int64_t* steps, int64_t* graphs_built, int64_t* graph_replays);

/* Admit a query; *query_id receives its id.  Errors: IM_EINVAL (J, K, graph),
 * IM_ENOMEM (no free slot or budget exceeded; nothing changed), IM_EDEVICE. */
im_status im_engine_submit(im_engine* e, const im_graph* g, int32_t J, uint64_t seed, int32_t K, int64_t* query_id);

/* Advance every running query by one stage (a few sweeps or cascade levels).
 * *n_running (optional) receives the number of queries still running. */
im_status im_engine_step(im_engine* e, int32_t* n_running);

/* Ids of finished queries (up to capacity of them in done_ids; *n_done = all). */
im_status im_engine_poll(im_engine* e, int64_t* done_ids, int32_t capacity, int32_t* n_done);

/* Results of a finished query (same meaning as im_select_seeds); the query's
 * device memory is released and its id becomes invalid.  IM_ESTATE if the
 * query has not finished. */
im_status im_engine_result(im_engine* e, int64_t query_id, int32_t* seeds_host, double* spread_out,
                           double* est_host, uint64_t* T_host, im_stats* stats_out);

/* Queries held, queries running, device bytes held and the budget. */
im_status im_engine_info(const im_engine* e, int32_t* n_queries, int32_t* n_running, uint64_t* bytes_used,
                         uint64_t* bytes_budget);

/* Device bytes a query (g, J, K) holds while admitted (0 for bad arguments). */
uint64_t im_query_footprint(const im_graph* g, int32_t J, int32_t K);

void im_engine_free(im_engine* e);

/* G independent queries in one engine, run to completion: seeds_out[i] is an
 * int32[K[i]] host buffer, spread_out (optional) double[G].  With 16 or more
 * queries the engine runs in graph mode (use_graphs = 1): its steps are
 * captured and replayed; in both modes the workgroups of each launch are split
 * among the queries on the device. */
im_status im_select_seeds_batch(int32_t G, const im_graph* const* graphs, const int32_t* J, const uint64_t* seed,
                                const int32_t* K, int32_t* const* seeds_out, double* spread_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* IMX_IM_H */
