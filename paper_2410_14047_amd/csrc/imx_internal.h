// Internal interfaces between the C-ABI host layer (api.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imx {

constexpr int kWaves = 4;             // waves per workgroup in the wave-per-task kernels
constexpr int kWG = 64 * kWaves;      // workgroup size
constexpr int kMaxJ = 4096;           // registers per vertex, upper bound
constexpr int kArgmaxBlocks = 1024;   // partial-argmax workgroups
constexpr int kBuckets = 1024;        // bucket table over the top bits of the 31-bit X values
constexpr int kBucketShift = 21;      // X >> 21 selects the bucket
// LDS words of the X values plus bucket table, padded to 16 bytes so that the
// per-wave and per-group areas after it keep 8- and 16-byte alignment.
constexpr int kTableWords = ((kBuckets + 1 + 3) / 4) * 4;

// Device view of a loaded graph and its work decomposition.
//   Out-tasks: every vertex u with out-degree > 0 owns the tasks
//   task_start[u] .. task_start[u+1]-1, each a run of at most `split`
//   consecutive out-arcs starting at task_e0[t].
//   In-tasks: the same over the reverse graph (in-arcs of v, sources in
//   in_col), runs of at most `in_split` in-arcs.
struct GraphDev {
    int64_t n, m;
    const int64_t* rowptr;        // [n+1]
    const int32_t* col;           // [m]
    const uint32_t* W;            // [m] 31-bit fixed-point thresholds
    const int32_t* task_u;        // [ntasks]
    const int64_t* task_e0;       // [ntasks]
    const uint32_t* task_len;     // [ntasks] arcs in the task; bit 31 set when u has several tasks
    const int32_t* task_start;    // [n+1]
    int64_t ntasks;
    int32_t split;
    const int64_t* in_rowptr;     // [n+1]
    const int32_t* in_col;        // [m] source of each in-arc
    const int32_t* in_task_v;     // [n_in_tasks]
    const int64_t* in_task_e0;    // [n_in_tasks]
    const int32_t* in_task_start; // [n+1]
    int64_t n_in_tasks;
    int32_t in_split;
};

// Device state of the propagation sweeps.  Sweep s reads chg[s&1] (rows that
// changed in sweep s-1) and the active task list act_tasks[s&1] (count
// act_count[s&3]); it writes chg[(s+1)&1], the in-tasks of its changed rows
// (chg_list, count chg_count[s&3]) and rows_changed[s&3].  The mark step of
// sweep s flags the sources of those in-arcs in act8 (plain byte stores), and
// the prep step of sweep s+1 compacts the flags into act_tasks[(s+1)&1] /
// act_count[(s+1)&3], clearing them.
struct SweepDev {
    int32_t* act_tasks[2];            // [ntasks] each
    uint32_t* act_count;              // [4]
    uint32_t* chg[2];                 // [ceil(n/32)] each
    uint8_t* act8;                    // [flag_bytes(n)] vertex activated for the next sweep; all 0 between sweeps
    int32_t* chg_list;                // [n_in_tasks]
    uint32_t* chg_count;              // [4]
    unsigned long long* rows_changed; // [4]
    uint32_t* dense;                  // [4] sweep s visits every task when dense[s&3] != 0
    uint32_t* conv;                   // first sweep of the build that changed no row (~0u: none yet);
                                      // kernels of later sweeps return at once
};

// Device state of the covering cascade (union-frontier BFS over tasks).
// Level t flags the vertices it newly covers in lv8 (plain byte stores); the
// compaction after level t turns the flags into frontier Q_{t+1} and the
// touched list, clearing them.
struct CascadeDev {
    int32_t* q[2];           // frontier out-task lists, capacity ntasks each
    uint32_t* qsize;         // ring of 4 list-size counters
    uint8_t* lv8;            // [flag_bytes(n)] covered at the current level; all 0 between levels
    int32_t* touched;        // [n] distinct vertices touched by this cascade
    uint32_t* ntouched;      // counter for `touched`
    uint32_t* touch_stamp;   // [n] id of the last cascade that touched v
    unsigned long long* T;   // covered (vertex, simulation) pairs
    uint32_t* level_end;     // first level of the cascade with an empty frontier (~0u: running)
};

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

// Packed propagation kernel: a wave takes pack_rows(J)
// tasks at once, staging kPackBytes of register rows (at least one row).
constexpr int kPackBytes = 2048;
__host__ __device__ inline int pack_rows(int J)
{
    const int p = kPackBytes / J;
    return p < 1 ? 1 : (p > 16 ? 16 : p);
}

// Per-vertex flag arrays are padded to whole 16-byte chunks.
inline int64_t flag_bytes(int64_t n) { return (n + 15) / 16 * 16; }

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

struct ArgmaxScratch {
    uint32_t* pJ;            // [kArgmaxBlocks]
    unsigned long long* pH;  // [kArgmaxBlocks]
    int32_t* pid;            // [kArgmaxBlocks]
};

// ---------------------------------------------------------------------------
// Batched launches.  One launch serves up to kMaxBatch queries: query i owns
// workgroups wg0[i] .. wg0[i+1]-1 and the argument record args[i] (an array
// in device memory).

constexpr int kMaxBatch = 64;

struct Batch {
    int nq;
    int wg0[kMaxBatch + 1];
};

struct FillArgs {
    uint8_t* M;
    int64_t n;
    int J;
    int first;  // fresh sketch: every register uncovered
    uint64_t seed;
};

struct PrepArgs {
    SweepDev s;
    const int32_t* task_start;  // [n+1] out-tasks of each vertex
    int64_t n;
    int64_t nwords;
    int sweep;
};

struct PropArgs {
    GraphDev g;
    const uint32_t* X;            // sorted values + bucket table
    int J;
    uint8_t* M;
    const int32_t* tasks;         // active tasks (nullptr: every task)
    const uint32_t* task_count;   // device count of `tasks`
    const uint32_t* chg_prev;
    uint32_t* chg_next;
    int32_t* chg_list;
    uint32_t* chg_count;
    const uint32_t* dense;        // nonzero: visit every task this sweep
    const uint32_t* conv;         // the build converged before this sweep when != ~0u
    unsigned long long* rows_changed;
    PropCounters* stats;          // instrumented variant only
    uint32_t* vstamp;             // instrumented variant only: [n] last launch id that counted row u
    uint32_t stamp_id;            // instrumented variant only: id of this launch (increasing)
};

struct MarkArgs {
    GraphDev g;
    SweepDev s;
    int sweep;
    int dense_div;  // next sweep visits every task when more than n / dense_div rows changed
};

struct EstArgs {
    const uint8_t* M;
    int64_t n;
    int J;
    uint32_t* Ju;
    unsigned long long* Hu;
};

struct ArgmaxArgs {
    const uint32_t* Ju;
    const unsigned long long* Hu;
    const uint8_t* is_seed;
    int64_t n;
    ArgmaxScratch am;
    int32_t* best;
    int nparts;  // workgroups of the partial pass for this query
};

struct SeedArgs {
    GraphDev g;
    const int32_t* best;
    int32_t k;
    uint8_t* M;
    int J;
    uint8_t* is_seed;
    int32_t* seeds;
    uint32_t* pickJ;
    unsigned long long* pickH;
    const uint32_t* Ju;
    const unsigned long long* Hu;
    CascadeDev c;
    uint32_t cascade_id;
};

struct LevelArgs {
    GraphDev g;
    const uint32_t* X;
    int J;
    uint8_t* M;
    CascadeDev c;
    int t;
};

struct LevelCompactArgs {
    const int32_t* task_start;  // [n+1]
    int64_t n;
    CascadeDev c;
    int t;                // the level whose flags are compacted into Q_{t+1}
    uint32_t cascade_id;
};

struct FinArgs {
    uint8_t* M;
    int J;
    uint32_t* Ju;
    unsigned long long* Hu;
    CascadeDev c;
};

int device_cu_count();
int propagate_group_size(int J, int requested);
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

}  // namespace imx
