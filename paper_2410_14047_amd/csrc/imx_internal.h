// Internal interfaces between the C-ABI host layer (api.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pack_layout.h"

namespace imx {

constexpr int kWaves = 4;             // waves per workgroup in the wave-per-task kernels
constexpr int kWG = 64 * kWaves;      // workgroup size
constexpr int kMaxJ = 4096;           // registers per vertex, upper bound
constexpr int kArgmaxBlocks = 1024;   // partial-argmax workgroups

// Pointers in the records below point to device memory.  A record has two
// views with one layout: the host view (G = false, plain pointers), which host
// code fills, and the kernels' view (G = true), whose pointers carry the
// global address space in device code.  Accesses through them compile to
// global_* instructions rather than flat_* ones; a flat access also counts
// against the LDS wait counter, so every wait for an LDS result would also
// wait for the global loads in flight and undo their prefetching.
template <class T, bool G>
struct dptr_s {
    using type = T*;
};
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
struct dptr_s<T, true> {
    using type = __attribute__((address_space(1))) T*;
};
#endif
template <class T, bool G>
using dptr = typename dptr_s<T, G>::type;
template <class T>
using gptr = dptr<T, true>;

// Device view of a loaded graph and its work decomposition.
//   Out-tasks: every vertex u with out-degree > 0 owns the tasks
//   task_start[u] .. task_start[u+1]-1, each a run of at most `split`
//   consecutive out-arcs starting at task_e0[t].
//   In-tasks: the same over the reverse graph (in-arcs of v, sources in
//   in_col), runs of at most `in_split` in-arcs.
template <bool G>
struct GraphDevT {
    int64_t n, m;
    dptr<const int64_t, G> rowptr;        // [n+1]
    dptr<const int32_t, G> col;           // [m]
    dptr<const uint32_t, G> W;            // [m] 31-bit fixed-point thresholds
    dptr<const int32_t, G> task_u;        // [ntasks]
    dptr<const int64_t, G> task_e0;       // [ntasks]
    dptr<const uint32_t, G> task_len;     // [ntasks] arcs in the task; bit 31 set when u has several tasks
    dptr<const int32_t, G> task_start;    // [n+1]
    int64_t ntasks;
    int32_t split;
    dptr<const int64_t, G> in_rowptr;     // [n+1]
    dptr<const int32_t, G> in_col;        // [m] source of each in-arc
    dptr<const int32_t, G> in_task_v;     // [n_in_tasks]
    dptr<const int64_t, G> in_task_e0;    // [n_in_tasks]
    dptr<const int32_t, G> in_task_start; // [n+1]
    int64_t n_in_tasks;
    int32_t in_split;
    // The task records again, ordered by descending arc count (ties by task
    // id): the order in which a sweep that visits every task deals them.
    dptr<const int32_t, G> dense_u;      // [ntasks]
    dptr<const int64_t, G> dense_e0;     // [ntasks]
    dptr<const uint32_t, G> dense_len;   // [ntasks]
};
using GraphDev = GraphDevT<false>;

// Device state of the propagation sweeps.  Sweep s reads chg[s&1] (rows that
// changed in sweep s-1) and the active task list act_tasks[s&1] (count
// act_count[s&3]); it writes chg[(s+1)&1], the in-tasks of its changed rows
// (chg_list, count chg_count[s&3]) and rows_changed[s&3].  The mark step of
// sweep s flags the sources of those in-arcs in act8 (plain byte stores), and
// the prep step of sweep s+1 compacts the flags into act_tasks[(s+1)&1] /
// act_count[(s+1)&3], clearing them.
template <bool G>
struct SweepDevT {
    dptr<int32_t, G> act_tasks[2];            // [ntasks] each
    dptr<uint32_t, G> act_count;              // [4]
    dptr<uint32_t, G> chg[2];                 // [ceil(n/32)] each
    dptr<uint8_t, G> act8;                    // [flag_bytes(n)] vertex activated for the next sweep; all 0 between sweeps
    dptr<uint8_t, G> act_blk;                 // [blk_bytes(n)] some vertex of the 1024-vertex block is flagged in act8
    dptr<int32_t, G> chg_list;                // [n_in_tasks]
    dptr<uint32_t, G> chg_count;              // [4]
    dptr<unsigned long long, G> rows_changed; // [4]
    dptr<uint32_t, G> dense;                  // [4] sweep s visits every task when dense[s&3] != 0
    dptr<uint32_t, G> conv;                   // first sweep of the build that changed no row (~0u: none yet);
                                      // kernels of later sweeps return at once
};
using SweepDev = SweepDevT<false>;

// Device state of the covering cascade (union-frontier BFS over tasks).
// Level t flags the vertices it newly covers in lv8 (plain byte stores); the
// compaction after level t turns the flags into frontier Q_{t+1} and the
// touched list, clearing them.
template <bool G>
struct CascadeDevT {
    dptr<int32_t, G> q[2];           // frontier out-task lists, capacity ntasks each
    dptr<uint32_t, G> qsize;         // ring of 4 list-size counters
    dptr<uint8_t, G> lv8;            // [flag_bytes(n)] covered at the current level; all 0 between levels
    dptr<uint8_t, G> lv_blk;         // [blk_bytes(n)] some vertex of the 1024-vertex block is flagged in lv8
    dptr<int32_t, G> touched;        // [n] distinct vertices touched by this cascade
    dptr<uint32_t, G> ntouched;      // counter for `touched`
    dptr<uint32_t, G> touch_stamp;   // [n] id of the last cascade that touched v
    dptr<unsigned long long, G> T;   // covered (vertex, simulation) pairs
    dptr<uint32_t, G> level_end;     // first level of the cascade with an empty frontier (~0u: running)
};
using CascadeDev = CascadeDevT<false>;

// Row-streaming kernels (fill, estimate) give each row an aligned group of L
// lanes, L the largest power of two not above min(64, J/16); each lane owns
// 16-byte chunks (16 registers) of the row, strided by L.
__host__ __device__ inline int row_lanes(int J)
{
    const int c = J / 16;
    return (c >= 64) ? 64 : (c >= 32) ? 32 : (c >= 16) ? 16 : (c >= 8) ? 8 : 4;
}

// Rows a lane group of the row-streaming kernels handles together (loads in flight).
constexpr int kRowBatch = 4;

// Packed propagation kernel: a wave takes pack_rows(J, pb) tasks at once,
// staging pb bytes of register rows (at least one row); pb = pack_bytes(),
// 1024, 2048 or 4096 (environment IMX_PACK_BYTES, read once).
int pack_bytes();
__host__ __device__ inline int pack_rows(int J, int pb)
{
    const int p = pb / J;
    return p < 1 ? 1 : (p > 16 ? 16 : p);
}

// Per-vertex flag arrays are padded to whole 16-byte chunks.
inline int64_t flag_bytes(int64_t n) { return (n + 15) / 16 * 16; }
// Flag arrays have a summary byte per block of kFlagBlock vertices (set
// with every flag of the block), so a compaction skips blocks without flags
// (frontiers of road-like graphs occupy few blocks).
constexpr int kFlagBlockShift = 10;
constexpr int kFlagBlock = 1 << kFlagBlockShift;
inline int64_t blk_bytes(int64_t n) { return flag_bytes((n + kFlagBlock - 1) / kFlagBlock); }

// Event counts of the instrumented propagation kernel (algorithmic traffic).
struct PropCounters {
    unsigned long long tasks;          // tasks visited
    unsigned long long rows_read;      // rows of u read (J bytes each)
    unsigned long long bytes_written;  // register bytes stored (changed 32-bit words x 4)
    unsigned long long arcs_scanned;   // arcs whose head id was read
    unsigned long long arcs_active;    // arcs whose head changed in the previous sweep
    unsigned long long sectors;        // distinct 64-byte sectors of head rows holding live registers
    unsigned long long rows_visited;   // distinct rows u with at least one arc whose head changed
    unsigned long long rows_changed;   // distinct rows u that changed
};

template <bool G>
struct ArgmaxScratchT {
    dptr<uint32_t, G> pJ;            // [kArgmaxBlocks]
    dptr<unsigned long long, G> pH;  // [kArgmaxBlocks]
    dptr<int32_t, G> pid;            // [kArgmaxBlocks]
    // Lazy selection: partial b is recomputed only when dirty[b] != 0, i.e.
    // when a vertex of its block changed its estimate terms or seed flag since
    // the partial was last computed (the cascade's finalize and the estimate
    // pass set the flags).  nullptr: every partial is recomputed.
    dptr<uint8_t, G> dirty = nullptr;  // [kArgmaxBlocks]
};
using ArgmaxScratch = ArgmaxScratchT<false>;

// ---------------------------------------------------------------------------
// Batched launches.  One launch serves up to kMaxBatch queries: query i owns
// workgroups wg0[i] .. wg0[i+1]-1 and the argument record args[i] (an array
// in device memory).  A record whose `active` member is 0 makes its
// workgroups return at once.

constexpr int kMaxBatch = 64;

struct Batch {
    int nq;
    int wg0[kMaxBatch + 1];
};

template <bool G>
struct FillArgsT {
    dptr<uint8_t, G> M;
    int64_t n;
    int J;
    int first;  // fresh sketch: every register uncovered
    uint64_t seed;
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using FillArgs = FillArgsT<false>;

template <bool G>
struct PrepArgsT {
    SweepDevT<G> s;
    dptr<const int32_t, G> task_start;  // [n+1] out-tasks of each vertex
    int64_t n;
    int64_t nwords;
    int sweep;
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using PrepArgs = PrepArgsT<false>;

template <bool G>
struct PropArgsT {
    GraphDevT<G> g;
    dptr<const uint32_t, G> X;            // sorted values + bucket table
    int J;
    dptr<uint8_t, G> M;
    dptr<const int32_t, G> tasks;         // active tasks (nullptr: every task)
    dptr<const uint32_t, G> task_count;   // device count of `tasks`
    dptr<const uint32_t, G> chg_prev;
    dptr<uint32_t, G> chg_next;
    dptr<int32_t, G> chg_list;
    dptr<uint32_t, G> chg_count;
    dptr<const uint32_t, G> dense;        // nonzero: visit every task this sweep
    dptr<const uint32_t, G> conv;         // the build converged before this sweep when != ~0u
    dptr<unsigned long long, G> rows_changed;
    dptr<PropCounters, G> stats;          // instrumented variant only
    dptr<uint32_t, G> vstamp;             // instrumented variant only: [n] last launch id that counted row u
    uint32_t stamp_id;            // instrumented variant only: id of this launch (increasing)
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using PropArgs = PropArgsT<false>;

template <bool G>
struct MarkArgsT {
    GraphDevT<G> g;
    SweepDevT<G> s;
    int sweep;
    int dense_div;  // next sweep visits every task when more than n / dense_div rows changed
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using MarkArgs = MarkArgsT<false>;

template <bool G>
struct EstArgsT {
    dptr<const uint8_t, G> M;
    int64_t n;
    int J;
    dptr<uint32_t, G> Ju;
    dptr<unsigned long long, G> Hu;
    dptr<uint8_t, G> am_dirty = nullptr;  // every partial of the lazy argmax becomes dirty (or nullptr)
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using EstArgs = EstArgsT<false>;

template <bool G>
struct ArgmaxArgsT {
    dptr<const uint32_t, G> Ju;
    dptr<const unsigned long long, G> Hu;
    dptr<const uint8_t, G> is_seed;
    int64_t n;
    ArgmaxScratchT<G> am;
    dptr<int32_t, G> best;
    int nparts;  // workgroups of the partial pass for this query
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using ArgmaxArgs = ArgmaxArgsT<false>;

template <bool G>
struct SeedArgsT {
    GraphDevT<G> g;
    dptr<const int32_t, G> best;
    int32_t k;
    dptr<uint8_t, G> M;
    int J;
    dptr<uint8_t, G> is_seed;
    dptr<int32_t, G> seeds;
    dptr<uint32_t, G> pickJ;
    dptr<unsigned long long, G> pickH;
    dptr<const uint32_t, G> Ju;
    dptr<const unsigned long long, G> Hu;
    CascadeDevT<G> c;
    uint32_t cascade_id;
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using SeedArgs = SeedArgsT<false>;

template <bool G>
struct LevelArgsT {
    GraphDevT<G> g;
    dptr<const uint32_t, G> X;
    int J;
    dptr<uint8_t, G> M;
    CascadeDevT<G> c;
    int t;
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using LevelArgs = LevelArgsT<false>;

template <bool G>
struct LevelCompactArgsT {
    dptr<const int32_t, G> task_start;  // [n+1]
    int64_t n;
    CascadeDevT<G> c;
    int t;                // the level whose flags are compacted into Q_{t+1}
    uint32_t cascade_id;
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using LevelCompactArgs = LevelCompactArgsT<false>;

template <bool G>
struct FinArgsT {
    dptr<uint8_t, G> M;
    int J;
    dptr<uint32_t, G> Ju;
    dptr<unsigned long long, G> Hu;
    CascadeDevT<G> c;
    dptr<uint8_t, G> am_dirty = nullptr;  // the lazy argmax's partial of every touched row becomes dirty (or nullptr)
    int nparts = 1;                       // partials of the query's argmax
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using FinArgs = FinArgsT<false>;

// Tail kernels: one workgroup per query runs many sweeps (or cascade levels)
// in a loop while the frontier stays small, instead of three (or two) grid-wide
// launches per sweep (level).  The next frontier's distinct vertices are
// collected in an LDS set, so neither a pass over per-vertex flags nor
// device-scope atomics are needed.  When the frontier grows past the limits
// the kernel hands the query back to the full-grid path in a state that path
// continues from.
// Why a tail launch stopped: it ran all its rounds (the frontier is still
// small), the build converged or the cascade ended, or the frontier grew
// past the limits (handed back).
constexpr uint32_t kTailStopRounds = 0, kTailStopDone = 1, kTailStopLarge = 2;
constexpr int kTailCap = 2048;             // distinct vertices of one frontier held in LDS
constexpr int kTailSlots = 2 * kTailCap;   // LDS set slots

template <bool G>
struct TailSweepArgsT {
    GraphDevT<G> g;
    dptr<const uint32_t, G> X;
    int J;
    dptr<uint8_t, G> M;
    SweepDevT<G> s;
    dptr<int32_t, G> chg_list2;  // [n_in_tasks] second in-task list; the tail alternates it with s.chg_list
    dptr<uint32_t, G> next;      // out: the sweep the full-grid path runs next
    int s0;                      // first sweep; its task list was compacted by the prep step of s0
    int rounds;                  // sweeps at most
    int dense_div;               // as for the mark step
    int64_t arcs_max;            // hand back when the changed rows have more in-arcs than this
    int64_t tasks_max;           // hand back when the next list has more tasks than this
    dptr<uint32_t, G> reason;    // out: why the launch stopped (kTailStop*)
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using TailSweepArgs = TailSweepArgsT<false>;

template <bool G>
struct TailLevelArgsT {
    GraphDevT<G> g;
    dptr<const uint32_t, G> X;
    int J;
    dptr<uint8_t, G> M;
    CascadeDevT<G> c;
    dptr<uint32_t, G> next;         // out: the level the full-grid path runs next
    dptr<uint32_t, G> cmp_pending;  // out: level whose flags the compaction must turn into Q_{t+1} (~0u: none)
    int t0;                         // first level (Q_{t0} built)
    int rounds;                     // levels at most
    uint32_t tasks_max;             // hand back frontiers of more tasks than this
    uint32_t cascade_id;
    dptr<uint32_t, G> reason;       // out: why the launch stopped (kTailStop*)
    int active = 1;  // 0: this query skips the launch (fixed launch sequences of the engine's graph mode)
};
using TailLevelArgs = TailLevelArgsT<false>;

int device_cu_count();
int propagate_group_size(int J, int requested);
int propagate_wg_threads(int requested);  // threads per workgroup of the propagation kernel chosen by `requested`
hipError_t propagate_full_grid(int maxJ, int gs, bool stats, int* grid);
hipError_t cascade_level_full_grid(int maxJ, int* grid);

hipError_t launch_thresholds(const float* p, uint32_t* W, int64_t m, hipStream_t st);
// X receives J sorted values followed by the kBuckets+1 entry bucket table.
hipError_t launch_sim_values(uint64_t seed, int J, uint32_t* X, hipStream_t st);
hipError_t launch_fill(const FillArgs* args, const Batch& B, hipStream_t st);
hipError_t launch_sweep_prep(const PrepArgs* args, const Batch& B, hipStream_t st);
hipError_t launch_propagate(const PropArgs* args, const Batch& B, int maxJ, int gs, bool stats, hipStream_t st);
hipError_t launch_mark(const MarkArgs* args, const Batch& B, hipStream_t st);
hipError_t launch_estimate(const EstArgs* args, const Batch& B, hipStream_t st);
hipError_t launch_argmax(const ArgmaxArgs* args, const Batch& partial, const Batch& final_, hipStream_t st);
hipError_t launch_cascade_seed(const SeedArgs* args, const Batch& B, hipStream_t st);
hipError_t launch_cascade_level(const LevelArgs* args, const Batch& B, int maxJ, hipStream_t st);
hipError_t launch_cascade_compact(const LevelCompactArgs* args, const Batch& B, hipStream_t st);
hipError_t launch_cascade_finalize(const FinArgs* args, const Batch& B, hipStream_t st);
// One workgroup per query (B.wg0[i] = i).
hipError_t launch_tail_sweeps(const TailSweepArgs* args, const Batch& B, int maxJ, hipStream_t st);
hipError_t launch_tail_levels(const TailLevelArgs* args, const Batch& B, int maxJ, hipStream_t st);

}  // namespace imx
