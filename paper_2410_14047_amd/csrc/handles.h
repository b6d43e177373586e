// Host-side handle types shared by the C-ABI files (api.cpp, engine.cpp).
#pragma once

#include "im.h"
#include "imx_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

namespace imx {

// Records the message of a failed call for im_last_error (per thread).
im_status set_error(im_status st, const std::string& msg);

// Process-wide profiling level (im_set_profiling).
int profiling_level();

#define IMX_HIP(expr)                                                                                      \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return ::imx::set_error(IM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

// Device memory source: hipMalloc/hipFree, or the hooks of im_set_allocator.
struct DeviceAllocator {
    im_alloc_fn alloc = nullptr;
    im_free_fn free_ = nullptr;
    void* ctx = nullptr;
};

// The hooks in effect now (a snapshot; im_set_allocator may change them).
DeviceAllocator current_allocator();

// One device buffer and the source that must free it.
struct DeviceBlock {
    void* ptr;
    DeviceAllocator from;
};

// Reported estimate of a pick (Eq. 7, harmonic form over uncovered
// registers): alpha_J * 2^33 * Ju^2 / (J * Hu), evaluated in one fixed order
// without contraction; 0 when Ju = 0.
double estimate_value(int J, uint32_t Ju, unsigned long long Hu);

hipError_t device_alloc(size_t bytes, DeviceBlock* out);
void device_free(const DeviceBlock& b);

// Device allocations of one handle; released together, each to its source.
struct Arena {
    std::vector<DeviceBlock> blocks;
    size_t bytes = 0;
    template <class T>
    hipError_t alloc(T** p, size_t count)
    {
        DeviceBlock b{};
        const size_t nb = std::max<size_t>(count * sizeof(T), 1);
        hipError_t e = device_alloc(nb, &b);
        if (e == hipSuccess) {
            blocks.push_back(b);
            bytes += nb;
            *p = static_cast<T*>(b.ptr);
        }
        return e;
    }
    void release()
    {
        for (const DeviceBlock& b : blocks) device_free(b);
        blocks.clear();
        bytes = 0;
    }
};

}  // namespace imx

struct im_graph {
    hipStream_t stream = nullptr;
    int64_t n = 0, m = 0;
    int64_t* rowptr = nullptr;
    int32_t* col = nullptr;
    uint32_t* W = nullptr;
    int32_t* task_u = nullptr;
    int64_t* task_e0 = nullptr;
    uint32_t* task_len = nullptr;
    int32_t* task_start = nullptr;
    int64_t ntasks = 0;
    int32_t split = 128;
    int64_t* in_rowptr = nullptr;
    int32_t* in_col = nullptr;
    int32_t* in_task_v = nullptr;
    int64_t* in_task_e0 = nullptr;
    int32_t* in_task_start = nullptr;
    int64_t n_in_tasks = 0;
    int32_t in_split = 256;
    int64_t max_out_deg = 0, max_in_deg = 0;
    int32_t* dense_u = nullptr;
    int64_t* dense_e0 = nullptr;
    uint32_t* dense_len = nullptr;
    imx::Arena arena;

    imx::GraphDev dev() const
    {
        return imx::GraphDev{n,          m,         rowptr,     col,           W,          task_u,
                             task_e0,    task_len,  task_start, ntasks,        split,      in_rowptr,
                             in_col,     in_task_v, in_task_e0, in_task_start, n_in_tasks, in_split,
                             dense_u,    dense_e0,  dense_len};
    }
};
