// Seed selection for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
// im_select_seeds_noalloc runs the same query as im_sketch_build followed by
// im_select_seeds (Alg. 4: fill and propagation to the fixed point, then K x
// [estimate, argmax, covering cascade, score, rebuild test]) with the same
// kernels, but its working buffers (simulation values, estimate terms,
// frontier lists and flags, cascade queues, argmax partials, status and
// argument records) live in one fixed device array, `scratch`, and the
// registers in a device buffer the caller passes.  No device or pinned host
// memory is allocated.
//
// `scratch` is a file-scope device array; each device the library runs on
// holds its own copy for the life of the process.  Host code never uses the
// array's name as an address: at a device's first call its address is taken
// with hipGetSymbolAddress (with that device current) and kept per device.
// Every call on one device shares that device's array; calls that overlap on
// one device (several host threads, or several streams) race and must be
// serialised by the caller.
#include "handles.h"

#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

namespace imx {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
constexpr int kRounds = 8;  // sweeps / cascade levels launched per host check

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mutex;
uint8_t* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch array, taken once per device.
im_status scratch_address(uint8_t** out)
{
    int dev = -1;
    IMX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(IM_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        IMX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(IM_EDEVICE, "scratch array has no device address");
        g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return IM_OK;
}

// Counters the host reads back after each batch of launches.
struct NaStatus {
    unsigned long long rows_changed[4];
    unsigned long long T;
    uint32_t qsize[4];
    uint32_t act_count[4];
    uint32_t chg_count[4];
    uint32_t dense[4];
    uint32_t ntouched;
    uint32_t conv;
    uint32_t level_end;
    uint32_t pad[3];
};

// Bump placement of buffers in the scratch array (256-byte aligned); only
// sizes are computed when base is null.
struct Carve {
    uint8_t* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += std::max<size_t>(count * sizeof(T), 1);
        return p;
    }
};

// Argument records of one batch of launches: at most kRounds x 3 records
// plus a few, each in its own 1 KiB slot.
constexpr size_t kArgSlots = kRounds * 3 + 8;
constexpr size_t kArgSlot = 1024;
static_assert(sizeof(PropArgs) <= kArgSlot && sizeof(SeedArgs) <= kArgSlot && sizeof(MarkArgs) <= kArgSlot &&
                  sizeof(LevelArgs) <= kArgSlot,
              "argument slot too small");

struct NaBuffers {
    NaStatus* status;
    uint8_t* args;
    uint32_t* X;
    uint32_t* Ju;
    unsigned long long* Hu;
    uint8_t* is_seed;
    int32_t* best;
    SweepDev sw;
    CascadeDev c;
    ArgmaxScratch am;
    int32_t* seeds;
    uint32_t* pickJ;
    unsigned long long* pickH;
};

size_t carve(uint8_t* base, const im_graph* g, int J, int K, NaBuffers* b)
{
    Carve C{base};
    const size_t n = (size_t)g->n, bmw = (n + 31) / 32;
    const size_t nt = (size_t)std::max<int64_t>(g->ntasks, 1), nit = (size_t)std::max<int64_t>(g->n_in_tasks, 1);
    b->status = C.take<NaStatus>(1);
    b->args = C.take<uint8_t>(kArgSlots * kArgSlot);
    b->X = C.take<uint32_t>((size_t)J + kTableWords);
    b->Ju = C.take<uint32_t>(n);
    b->Hu = C.take<unsigned long long>(n);
    b->is_seed = C.take<uint8_t>(n);
    b->best = C.take<int32_t>(1);
    b->sw.chg[0] = C.take<uint32_t>(bmw);
    b->sw.chg[1] = C.take<uint32_t>(bmw);
    b->sw.act8 = C.take<uint8_t>((size_t)flag_bytes((int64_t)n));
    b->sw.act_tasks[0] = C.take<int32_t>(nt);
    b->sw.act_tasks[1] = C.take<int32_t>(nt);
    b->sw.chg_list = C.take<int32_t>(nit);
    b->c.q[0] = C.take<int32_t>(nt);
    b->c.q[1] = C.take<int32_t>(nt);
    b->c.lv8 = C.take<uint8_t>((size_t)flag_bytes((int64_t)n));
    b->c.touched = C.take<int32_t>(n);
    b->c.touch_stamp = C.take<uint32_t>(n);
    b->am.pJ = C.take<uint32_t>(kArgmaxBlocks);
    b->am.pH = C.take<unsigned long long>(kArgmaxBlocks);
    b->am.pid = C.take<int32_t>(kArgmaxBlocks);
    b->seeds = C.take<int32_t>((size_t)K);
    b->pickJ = C.take<uint32_t>((size_t)K);
    b->pickH = C.take<unsigned long long>((size_t)K);
    b->sw.act_blk = C.take<uint8_t>((size_t)blk_bytes((int64_t)n));
    b->c.lv_blk = C.take<uint8_t>((size_t)blk_bytes((int64_t)n));
    if (base) {
        NaStatus* S = b->status;
        b->sw.rows_changed = S->rows_changed;
        b->sw.act_count = S->act_count;
        b->sw.chg_count = S->chg_count;
        b->sw.dense = S->dense;
        b->sw.conv = &S->conv;
        b->c.level_end = &S->level_end;
        b->c.qsize = S->qsize;
        b->c.T = &S->T;
        b->c.ntouched = &S->ntouched;
    }
    return C.off;
}

Batch one_query(int64_t want, int64_t cap)
{
    Batch B{};
    B.nq = 1;
    B.wg0[0] = 0;
    int64_t w = std::max<int64_t>(want, 1);
    if (cap > 0) w = std::min(w, cap);
    B.wg0[1] = (int)w;
    return B;
}

// Host staging of one batch's argument records (per device; calls on one
// device are serialised by contract) and their copy into the scratch slots.
struct ArgStage {
    uint8_t host[kArgSlots * kArgSlot];
    size_t used = 0;     // slots staged since the last wait
    size_t flushed = 0;  // slots of those already copied to the device
};
ArgStage g_stage[kMaxDevices];

template <class A>
const A* stage(ArgStage& S, uint8_t* dev_slots, const A& rec)
{
    if (S.used >= kArgSlots) return nullptr;
    std::memcpy(S.host + S.used * kArgSlot, &rec, sizeof(A));
    return reinterpret_cast<const A*>(dev_slots + (S.used++) * kArgSlot);
}

struct Run {
    const im_graph* g;
    int J, K;
    uint64_t seed;
    uint8_t* M;
    hipStream_t st;
    NaBuffers b;
    ArgStage* S;
    int cus;
    NaStatus host_status;

    hipError_t flush_args()
    {
        hipError_t e = hipSuccess;
        if (S->used > S->flushed)
            e = hipMemcpyAsync(b.args + S->flushed * kArgSlot, S->host + S->flushed * kArgSlot,
                               (S->used - S->flushed) * kArgSlot, hipMemcpyHostToDevice, st);
        S->flushed = S->used;
        return e;
    }
    // Copies the status record back and waits for the batch (the staging
    // area may be reused afterwards).
    hipError_t sync_status()
    {
        hipError_t e = hipMemcpyAsync(&host_status, b.status, sizeof(NaStatus), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        S->used = S->flushed = 0;
        return e;
    }

    // Fill (Alg. 1), then sweeps of Alg. 2 until one changes no register,
    // then the estimate terms of every row (Eq. 7).
    im_status build(bool fresh, int* sweeps_out)
    {
        {
            const int64_t rows_per_wg = 256 / row_lanes(J);
            const FillArgs* fa = stage(*S, b.args, FillArgs{M, g->n, J, fresh ? 1 : 0, seed});
            if (!fa) return set_error(IM_EINVAL, "argument slots exhausted");
            IMX_HIP(flush_args());
            IMX_HIP(launch_fill(fa, one_query(std::min<int64_t>(cus * 16, (g->n + rows_per_wg - 1) / rows_per_wg), 0), st));
        }
        int full = 0;
        IMX_HIP(propagate_full_grid(J, 0, false, &full));
        const GraphDev gd = g->dev();
        const int lanes = propagate_group_size(J, 0), thr = propagate_wg_threads(0);
        for (int sweep = 0;; sweep += kRounds) {
            const PrepArgs* pa[kRounds];
            const PropArgs* ra[kRounds];
            const MarkArgs* ma[kRounds];
            for (int r = 0; r < kRounds; ++r) {
                const int s = sweep + r;
                pa[r] = stage(*S, b.args, PrepArgs{b.sw, g->task_start, g->n, (g->n + 31) / 32, s});
                ra[r] = stage(*S, b.args,
                              PropArgs{gd, b.X, J, M, s == 0 ? nullptr : b.sw.act_tasks[s & 1], &b.sw.act_count[s & 3],
                                       b.sw.chg[s & 1], b.sw.chg[(s + 1) & 1], b.sw.chg_list, &b.sw.chg_count[s & 3],
                                       &b.sw.dense[s & 3], b.sw.conv, &b.sw.rows_changed[s & 3], nullptr, nullptr, 0u});
                ma[r] = stage(*S, b.args, MarkArgs{gd, b.sw, s, 16});
                if (!pa[r] || !ra[r] || !ma[r]) return set_error(IM_EINVAL, "argument slots exhausted");
            }
            IMX_HIP(flush_args());
            for (int r = 0; r < kRounds; ++r) {
                IMX_HIP(launch_sweep_prep(pa[r], one_query(std::min<int64_t>(cus * 4, (g->n + 16 * kWG - 1) / (16 * kWG)), 0), st));
                IMX_HIP(launch_propagate(ra[r], one_query((g->ntasks * lanes + thr - 1) / thr, full), J, 0, false, st));
                IMX_HIP(launch_mark(ma[r], one_query(std::min<int64_t>(cus * 4, (g->n_in_tasks + kWaves - 1) / kWaves), cus * 4), st));
            }
            IMX_HIP(sync_status());
            if (host_status.conv != ~0u) {
                *sweeps_out = (int)host_status.conv + 1;
                break;
            }
            if (sweep > g->n + 2) return set_error(IM_EDEVICE, "propagation did not converge");
        }
        const int64_t rows_per_wg = kWG / row_lanes(J) * kRowBatch;
        const EstArgs* ea = stage(*S, b.args, EstArgs{M, g->n, J, b.Ju, b.Hu});
        IMX_HIP(flush_args());
        IMX_HIP(launch_estimate(ea, one_query(std::min<int64_t>(cus * 16, (g->n + rows_per_wg - 1) / rows_per_wg), 0), st));
        IMX_HIP(sync_status());
        return IM_OK;
    }

    // Pick k: exact argmax, then the covering cascade (Alg. 3) level by level
    // until a level is empty, then the finalize pass (markers to 0, estimate
    // terms of touched rows, T).  Returns T after the cascade.
    im_status pick(int k, uint32_t cascade_id, uint64_t* T)
    {
        int full_level = 0;
        IMX_HIP(cascade_level_full_grid(J, &full_level));
        const GraphDev gd = g->dev();
        const int nparts = std::max<int>(1, (int)std::min<int64_t>(kArgmaxBlocks, (g->n + 255) / 256));
        const ArgmaxArgs* aa = stage(*S, b.args, ArgmaxArgs{b.Ju, b.Hu, b.is_seed, g->n, b.am, b.best, nparts});
        const SeedArgs* sa = stage(*S, b.args,
                                   SeedArgs{gd, b.best, k, M, J, b.is_seed, b.seeds, b.pickJ, b.pickH, b.Ju, b.Hu, b.c,
                                            cascade_id});
        if (!aa || !sa) return set_error(IM_EINVAL, "argument slots exhausted");
        IMX_HIP(flush_args());
        Batch fin{};
        fin.nq = 1;
        fin.wg0[0] = 0;
        fin.wg0[1] = 1;
        IMX_HIP(launch_argmax(aa, one_query(nparts, 0), fin, st));
        IMX_HIP(launch_cascade_seed(sa, one_query(1, 0), st));
        IMX_HIP(sync_status());
        for (int level = 1;; level += kRounds) {
            const LevelArgs* la[kRounds];
            const LevelCompactArgs* ca[kRounds];
            for (int r = 0; r < kRounds; ++r) {
                la[r] = stage(*S, b.args, LevelArgs{gd, b.X, J, M, b.c, level + r});
                ca[r] = stage(*S, b.args, LevelCompactArgs{g->task_start, g->n, b.c, level + r, cascade_id});
                if (!la[r] || !ca[r]) return set_error(IM_EINVAL, "argument slots exhausted");
            }
            const FinArgs* fa = stage(*S, b.args, FinArgs{M, J, b.Ju, b.Hu, b.c});
            if (!fa) return set_error(IM_EINVAL, "argument slots exhausted");
            IMX_HIP(flush_args());
            for (int r = 0; r < kRounds; ++r) {
                IMX_HIP(launch_cascade_level(la[r], one_query((g->ntasks + kWaves - 1) / kWaves, full_level), J, st));
                IMX_HIP(launch_cascade_compact(ca[r], one_query(std::min<int64_t>(cus * 4, (g->n + 16 * kWG - 1) / (16 * kWG)), 0), st));
            }
            IMX_HIP(launch_cascade_finalize(fa, one_query(std::min<int64_t>(cus * 8, (g->n + 4 * kWaves - 1) / (4 * kWaves)), 0), st));
            IMX_HIP(sync_status());
            if (host_status.level_end != ~0u) {
                *T = host_status.T;
                return IM_OK;
            }
            if (level > g->n + 8) return set_error(IM_EDEVICE, "cascade did not terminate");
        }
    }
};

}  // namespace

size_t noalloc_scratch_bytes(const im_graph* g, int J, int K)
{
    NaBuffers b{};
    return carve(nullptr, g, J, K, &b);
}

}  // namespace imx

extern "C" {

im_status im_select_seeds_noalloc(const im_graph* g, int32_t J, uint64_t seed, int32_t K, uint8_t* registers_dev,
                                  int32_t* seeds_host, double* spread_out, double* est_host, void* stream)
{
    using namespace imx;
    if (!g || !registers_dev || !seeds_host) return set_error(IM_EINVAL, "NULL argument");
    if (J < 64 || J > kMaxJ || J % 64 != 0) return set_error(IM_EINVAL, "J must be a multiple of 64 in [64, 4096]");
    if (K < 1 || K > g->n) return set_error(IM_EINVAL, "K must be in [1, n]");
    const size_t need = noalloc_scratch_bytes(g, J, K);
    if (need > kScratchBytes)
        return set_error(IM_EINVAL, "query needs " + std::to_string(need) + " bytes of scratch; the no-allocation entry "
                                    "point holds at most " + std::to_string(kScratchBytes));
    uint8_t* base = nullptr;
    if (im_status e = scratch_address(&base)) return e;
    int dev = 0;
    IMX_HIP(hipGetDevice(&dev));

    Run R{};
    R.g = g;
    R.J = J;
    R.K = K;
    R.seed = seed;
    R.M = registers_dev;
    R.st = static_cast<hipStream_t>(stream);
    R.S = &g_stage[dev];
    R.S->used = R.S->flushed = 0;
    R.cus = device_cu_count();
    carve(base, g, J, K, &R.b);
    // what must start at zero: status record, seed flags, activation and level
    // flags, cascade stamps
    IMX_HIP(hipMemsetAsync(R.b.status, 0, sizeof(NaStatus), R.st));
    IMX_HIP(hipMemsetAsync(R.b.is_seed, 0, (size_t)g->n, R.st));
    IMX_HIP(hipMemsetAsync(R.b.sw.act8, 0, (size_t)flag_bytes(g->n), R.st));
    IMX_HIP(hipMemsetAsync(R.b.c.lv8, 0, (size_t)flag_bytes(g->n), R.st));
    IMX_HIP(hipMemsetAsync(R.b.c.touch_stamp, 0, sizeof(uint32_t) * (size_t)g->n, R.st));
    IMX_HIP(hipMemsetAsync(R.b.sw.act_blk, 0, (size_t)blk_bytes(g->n), R.st));
    IMX_HIP(hipMemsetAsync(R.b.c.lv_blk, 0, (size_t)blk_bytes(g->n), R.st));
    IMX_HIP(launch_sim_values(seed, J, R.b.X, R.st));

    int sweeps = 0;
    if (im_status e = R.build(true, &sweeps)) return e;
    uint64_t T = 0, T_old = 0;
    for (int k = 0; k < K; ++k) {
        if (im_status e = R.pick(k, (uint32_t)(k + 1), &T)) return e;
        if (k + 1 < K && 100 * (T - T_old) > T) {  // error-adaptive rebuild (Alg. 4)
            T_old = T;
            if (im_status e = R.build(false, &sweeps)) return e;
        }
    }
    uint32_t hJ[1];
    unsigned long long hH[1];
    for (int k = 0; k < K; ++k) {
        int32_t s = -1;
        IMX_HIP(hipMemcpyAsync(&s, R.b.seeds + k, sizeof(int32_t), hipMemcpyDeviceToHost, R.st));
        IMX_HIP(hipMemcpyAsync(hJ, R.b.pickJ + k, sizeof(uint32_t), hipMemcpyDeviceToHost, R.st));
        IMX_HIP(hipMemcpyAsync(hH, R.b.pickH + k, sizeof(unsigned long long), hipMemcpyDeviceToHost, R.st));
        IMX_HIP(hipStreamSynchronize(R.st));
        if (s < 0) return set_error(IM_EDEVICE, "argmax found no candidate");
        seeds_host[k] = s;
        if (est_host) est_host[k] = estimate_value(J, hJ[0], hH[0]);
    }
    if (spread_out) *spread_out = (double)T / (double)J;
    return IM_OK;
}

}  // extern "C"
