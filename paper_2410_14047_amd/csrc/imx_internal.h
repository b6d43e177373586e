// Internal interfaces between the C-ABI host layer (api.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imx {

constexpr int kWaves = 4;             // waves per workgroup in the wave-per-row kernels
constexpr int kWG = 64 * kWaves;      // workgroup size
constexpr int kMaxJ = 4096;           // registers per vertex, upper bound
constexpr int kArgmaxBlocks = 1024;   // partial-argmax workgroups

// Device view of a loaded graph plus its propagation work list: every vertex
// with out-degree > 0 owns ceil(deg / split) tasks, each a run of at most
// `split` consecutive out-arcs.
struct GraphDev {
    int64_t n, m;
    const int64_t* rowptr;   // [n+1]
    const int32_t* col;      // [m]
    const uint32_t* W;       // [m] 31-bit fixed-point thresholds
    const int32_t* task_u;   // [ntasks] source vertex of the task
    const int64_t* task_e0;  // [ntasks] first arc of the task
    int64_t ntasks;
    int32_t split;           // max arcs per task
};

// Device state of the covering cascade (union-frontier BFS).
struct CascadeDev {
    int32_t* q[2];           // frontier queues, capacity n each
    uint32_t* qsize;         // ring of 4 queue-size counters
    uint32_t* stamp;         // [n] id of the last frontier v was appended to
    int32_t* touched;        // [n] distinct vertices touched by this cascade
    uint32_t* ntouched;      // counter for `touched`
    uint32_t* touch_stamp;   // [n] id of the last cascade that touched v
    unsigned long long* T;   // covered (vertex, simulation) pairs
};

struct ArgmaxScratch {
    uint32_t* pJ;            // [kArgmaxBlocks]
    unsigned long long* pH;  // [kArgmaxBlocks]
    int32_t* pid;            // [kArgmaxBlocks]
};

hipError_t launch_thresholds(const float* p, uint32_t* W, int64_t m, hipStream_t st);
hipError_t launch_sim_values(uint64_t seed, int J, uint32_t* X, hipStream_t st);
hipError_t launch_fill(uint8_t* M, int64_t n, int J, uint64_t seed, bool first, hipStream_t st);
hipError_t launch_propagate(const GraphDev& g, const uint32_t* X, int J, uint8_t* M, const uint32_t* chg_prev,
                            uint32_t* chg_next, unsigned long long* changed, hipStream_t st);
hipError_t launch_estimate(const uint8_t* M, int64_t n, int J, uint32_t* Ju, unsigned long long* Hu,
                           hipStream_t st);
hipError_t launch_argmax(const uint32_t* Ju, const unsigned long long* Hu, const uint8_t* is_seed, int64_t n,
                         const ArgmaxScratch& s, int32_t* best, hipStream_t st);
hipError_t launch_cascade_seed(const int32_t* best, int32_t k, uint8_t* M, int J, uint8_t* is_seed,
                               int32_t* seeds, uint32_t* pickJ, unsigned long long* pickH, const uint32_t* Ju,
                               const unsigned long long* Hu, const CascadeDev& c, uint32_t cascade_id,
                               uint32_t level_id1, hipStream_t st);
hipError_t launch_cascade_level(const GraphDev& g, const uint32_t* X, int J, uint8_t* M, const CascadeDev& c,
                                int t, uint32_t level_id, uint32_t cascade_id, hipStream_t st);
hipError_t launch_cascade_finalize(uint8_t* M, int J, uint32_t* Ju, unsigned long long* Hu, const CascadeDev& c,
                                   hipStream_t st);

}  // namespace imx
