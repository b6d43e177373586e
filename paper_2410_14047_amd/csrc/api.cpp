// C-ABI host layer of libimx.so: argument validation, device memory, the
// build / select drivers (Alg. 4 on one device) and the parity hooks.
// Every step of the method runs in the kernels of kernels.hip; this file only
// orders launches and moves the few scalars the host decisions need.
#include "im.h"
#include "imx_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

im_status fail(im_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

#define IMX_HIP(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(IM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device allocations of one handle; released together.
struct Arena {
    std::vector<void*> ptrs;
    template <class T>
    hipError_t alloc(T** p, size_t count)
    {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 1));
        if (e == hipSuccess) {
            ptrs.push_back(q);
            *p = static_cast<T*>(q);
        }
        return e;
    }
    void release()
    {
        for (void* p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
};

int default_split()
{
    const char* s = std::getenv("IMX_SPLIT");
    int v = s ? std::atoi(s) : 128;
    return (v >= 16 && v < (1 << 30)) ? v : 128;
}

// Lane-group size of the propagation kernel: full waves for the first sweep
// after a fill (every arc active, long runs of work per task), small groups
// for frontier sweeps (few active arcs per task, many tasks in flight).
int group_size_for(int sweep)
{
    const char* s = std::getenv(sweep == 0 ? "IMX_GROUP_FIRST" : "IMX_GROUP");
    const int dflt = 64;
    return s ? std::atoi(s) : dflt;
}

constexpr int kSweepBatch = 4;  // sweeps launched between host checks
constexpr int kLevelBatch = 4;  // cascade levels launched between host checks

std::atomic<int> g_profiling{0};

}  // namespace

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
    int32_t split = 512;
    int64_t* in_rowptr = nullptr;
    int32_t* in_col = nullptr;
    int32_t* in_task_v = nullptr;
    int64_t* in_task_e0 = nullptr;
    int32_t* in_task_start = nullptr;
    int64_t n_in_tasks = 0;
    int32_t in_split = 256;
    Arena arena;

    imx::GraphDev dev() const
    {
        return imx::GraphDev{n,          m,         rowptr,     col,           W,          task_u,
                             task_e0,    task_len,  task_start, ntasks,        split,      in_rowptr,
                             in_col,     in_task_v, in_task_e0, in_task_start, n_in_tasks, in_split};
    }
};

struct im_sketch {
    const im_graph* g = nullptr;
    hipStream_t stream = nullptr;
    int32_t J = 0;
    uint64_t seed = 0;
    uint8_t* M = nullptr;
    uint32_t* X = nullptr;
    uint32_t* Ju = nullptr;
    unsigned long long* Hu = nullptr;
    imx::SweepDev sw{};
    uint8_t* is_seed = nullptr;
    int32_t* best = nullptr;
    imx::CascadeDev casc{};
    imx::ArgmaxScratch am{};
    uint32_t cascade_id = 0;
    uint32_t level_base = 0;
    bool selected = false;
    im_stats st{};
    imx::PropCounters* pc = nullptr;      // instrumented-kernel counters (profiling 2)
    int profiling = 0;
    unsigned long long* h_ctr = nullptr;  // pinned
    uint32_t* h_qs = nullptr;             // pinned
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t evk[2 * kSweepBatch] = {};  // per-launch propagation timing
    Arena arena;

    ~im_sketch()
    {
        arena.release();
        if (h_ctr) (void)hipHostFree(h_ctr);
        if (h_qs) (void)hipHostFree(h_qs);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : evk)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

im_status check_device()
{
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || cnt < 1) return fail(IM_EDEVICE, "no HIP device available");
    return IM_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
}

// Fill (Alg. 1) then propagation sweeps (Alg. 2) until a sweep changes no
// register, then the estimate terms.  `first` = fresh sketch.
im_status run_build(im_sketch* s, bool first, int32_t* sweeps_out)
{
    const im_graph* g = s->g;
    const size_t bm_bytes = (size_t)((g->n + 31) / 32) * 4;
    hipStream_t st = s->stream;
    IMX_HIP(imx::launch_fill(s->M, g->n, s->J, s->seed, first, st));
    IMX_HIP(hipMemsetAsync(s->sw.chg[0], 0xff, bm_bytes, st));  // every row counts as changed
    if (s->pc) IMX_HIP(hipMemsetAsync(s->pc, 0, sizeof(imx::PropCounters), st));
    IMX_HIP(hipEventRecord(s->ev[2], st));
    int64_t sweeps = 0, launches = 0;
    bool done = false;
    const imx::GraphDev gd = g->dev();
    int sweep = 0;
    while (!done) {
        for (int b = 0; b < kSweepBatch; ++b, ++sweep) {
            IMX_HIP(imx::launch_sweep_prep(s->sw, g->n, sweep, st));
            IMX_HIP(hipEventRecord(s->evk[2 * b], st));
            IMX_HIP(imx::launch_propagate(gd, s->X, s->J, s->M, s->sw, sweep, group_size_for(sweep), s->pc, st));
            IMX_HIP(hipEventRecord(s->evk[2 * b + 1], st));
            IMX_HIP(imx::launch_mark(gd, s->sw, sweep, st));
        }
        IMX_HIP(hipMemcpyAsync(s->h_ctr, s->sw.rows_changed, sizeof(unsigned long long) * 4, hipMemcpyDeviceToHost,
                               st));
        IMX_HIP(hipStreamSynchronize(st));
        for (int b = 0; b < kSweepBatch; ++b) {
            s->st.prop_kernel_ms += elapsed(s->evk[2 * b], s->evk[2 * b + 1]);
            ++launches;
        }
        for (int b = 0; b < kSweepBatch; ++b) {
            ++sweeps;
            if (s->h_ctr[(sweep - kSweepBatch + b) & 3] == 0) {
                done = true;
                break;
            }
        }
        if (!done && sweeps > g->n + 2) return fail(IM_EDEVICE, "propagation did not converge");
    }
    IMX_HIP(hipEventRecord(s->ev[3], st));
    IMX_HIP(imx::launch_estimate(s->M, g->n, s->J, s->Ju, s->Hu, st));
    IMX_HIP(hipStreamSynchronize(st));
    s->st.prop_launches += launches;
    if (s->pc) {
        imx::PropCounters c{};
        IMX_HIP(hipMemcpyAsync(&c, s->pc, sizeof(c), hipMemcpyDeviceToHost, st));
        IMX_HIP(hipStreamSynchronize(st));
        s->st.prop_tasks += (int64_t)c.tasks;
        s->st.prop_rows_read += (int64_t)c.rows_read;
        s->st.prop_bytes_written += (int64_t)c.bytes_written;
        s->st.prop_arcs_scanned += (int64_t)c.arcs_scanned;
        s->st.prop_arcs_active += (int64_t)c.arcs_active;
        s->st.prop_sectors += (int64_t)c.sectors;
        s->st.prop_alg_bytes += 28.0 * c.tasks + 4.0 * c.arcs_scanned + 4.0 * c.arcs_active + 64.0 * c.sectors +
                                (double)s->J * c.rows_read + (double)c.bytes_written +
                                (double)((g->n + 31) / 32) * 4.0 * 2.0 * launches;
    }
    s->st.propagate_ms += elapsed(s->ev[2], s->ev[3]);
    s->st.total_sweeps += sweeps;
    if (sweeps_out) *sweeps_out = (int32_t)sweeps;
    return IM_OK;
}

}  // namespace

extern "C" {

const char* im_last_error(void) { return g_err.c_str(); }

im_status im_version(int32_t* major, int32_t* minor)
{
    if (major) *major = 0;
    if (minor) *minor = 1;
    return IM_OK;
}

im_status im_set_profiling(int32_t level)
{
    if (level != 0 && level != 2) return fail(IM_EINVAL, "profiling level must be 0 or 2");
    g_profiling.store(level);
    return IM_OK;
}

im_status im_graph_load(int64_t n, int64_t m, const int64_t* rowptr_host, const int32_t* col_host,
                        const float* p_host, void* stream, im_graph** out)
{
    if (!out) return fail(IM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(IM_EINVAL, "n must be in [1, 2^31)");
    if (m < 0 || m >= (int64_t(1) << 40)) return fail(IM_EINVAL, "m must be in [0, 2^40)");
    if (!rowptr_host || (m > 0 && (!col_host || !p_host))) return fail(IM_EINVAL, "NULL array");
    if (rowptr_host[0] != 0) return fail(IM_EINVAL, "rowptr[0] != 0");
    if (rowptr_host[n] != m) return fail(IM_EINVAL, "rowptr[n] != m");
    for (int64_t u = 0; u < n; ++u) {
        const int64_t b = rowptr_host[u], e = rowptr_host[u + 1];
        if (e < b) return fail(IM_EINVAL, "rowptr decreases at vertex " + std::to_string(u));
        for (int64_t i = b; i < e; ++i) {
            const int32_t v = col_host[i];
            if (v < 0 || v >= n) return fail(IM_EINVAL, "col out of range at arc " + std::to_string(i));
            if (i > b && v <= col_host[i - 1])
                return fail(IM_EINVAL, "col not strictly increasing within row at arc " + std::to_string(i));
            const float p = p_host[i];
            if (!(p >= 0.0f && p <= 1.0f)) return fail(IM_EINVAL, "p outside [0,1] at arc " + std::to_string(i));
        }
    }
    if (im_status e = check_device()) return e;

    const int split = default_split();
    const int in_split = 256;
    std::vector<int32_t> tu, ts(n + 1);
    std::vector<int64_t> te;
    std::vector<uint32_t> tl;
    for (int64_t u = 0; u < n; ++u) {
        ts[u] = (int32_t)tu.size();
        const int64_t deg = rowptr_host[u + 1] - rowptr_host[u];
        for (int64_t e0 = rowptr_host[u]; e0 < rowptr_host[u + 1]; e0 += split) {
            tu.push_back((int32_t)u);
            te.push_back(e0);
            const int64_t len = std::min<int64_t>(split, rowptr_host[u + 1] - e0);
            tl.push_back((uint32_t)len | (deg > split ? 0x80000000u : 0u));
        }
    }
    ts[n] = (int32_t)tu.size();
    if ((int64_t)tu.size() >= (int64_t(1) << 31)) return fail(IM_EINVAL, "too many propagation tasks");
    // reverse graph: in-arcs of every vertex, sources ascending
    std::vector<int64_t> irp(n + 1, 0);
    for (int64_t e = 0; e < m; ++e) ++irp[col_host[e] + 1];
    for (int64_t v = 0; v < n; ++v) irp[v + 1] += irp[v];
    std::vector<int32_t> icol(m);
    {
        std::vector<int64_t> pos(irp.begin(), irp.end() - 1);
        for (int64_t u = 0; u < n; ++u)
            for (int64_t e = rowptr_host[u]; e < rowptr_host[u + 1]; ++e) icol[pos[col_host[e]]++] = (int32_t)u;
    }
    std::vector<int32_t> itv, its(n + 1);
    std::vector<int64_t> ite;
    for (int64_t v = 0; v < n; ++v) {
        its[v] = (int32_t)itv.size();
        for (int64_t e0 = irp[v]; e0 < irp[v + 1]; e0 += in_split) {
            itv.push_back((int32_t)v);
            ite.push_back(e0);
        }
    }
    its[n] = (int32_t)itv.size();

    size_t need = sizeof(int64_t) * (n + 1) * 2 + (size_t)m * 16 + tu.size() * 12 + itv.size() * 12 + (size_t)n * 8;
    size_t free_b = 0, total_b = 0;
    IMX_HIP(hipMemGetInfo(&free_b, &total_b));
    if (need + (64u << 20) > free_b) return fail(IM_ENOMEM, "graph does not fit in device memory");

    im_graph* g = new im_graph();
    g->stream = static_cast<hipStream_t>(stream);
    g->n = n;
    g->m = m;
    g->split = split;
    g->ntasks = (int64_t)tu.size();
    g->in_split = in_split;
    g->n_in_tasks = (int64_t)itv.size();
    float* p_dev = nullptr;
    auto cleanup = [&](im_status st, const std::string& msg) {
        if (p_dev) (void)hipFree(p_dev);
        g->arena.release();
        delete g;
        return fail(st, msg);
    };
    Arena& A = g->arena;
    if (A.alloc(&g->rowptr, n + 1) || A.alloc(&g->col, m) || A.alloc(&g->W, m) || A.alloc(&g->task_u, tu.size()) ||
        A.alloc(&g->task_e0, te.size()) || A.alloc(&g->task_len, tl.size()) || A.alloc(&g->task_start, n + 1) || A.alloc(&g->in_rowptr, n + 1) ||
        A.alloc(&g->in_col, m) || A.alloc(&g->in_task_v, itv.size()) || A.alloc(&g->in_task_e0, ite.size()) ||
        A.alloc(&g->in_task_start, n + 1) || hipMalloc(&p_dev, std::max<size_t>(m * sizeof(float), 1)) != hipSuccess)
        return cleanup(IM_ENOMEM, "device allocation failed");
    hipStream_t st = g->stream;
    hipError_t e = hipMemcpyAsync(g->rowptr, rowptr_host, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && m) e = hipMemcpyAsync(g->col, col_host, sizeof(int32_t) * m, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && m) e = hipMemcpyAsync(p_dev, p_host, sizeof(float) * m, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !tu.empty())
        e = hipMemcpyAsync(g->task_u, tu.data(), sizeof(int32_t) * tu.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !te.empty())
        e = hipMemcpyAsync(g->task_e0, te.data(), sizeof(int64_t) * te.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !tl.empty())
        e = hipMemcpyAsync(g->task_len, tl.data(), sizeof(uint32_t) * tl.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->task_start, ts.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->in_rowptr, irp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && m)
        e = hipMemcpyAsync(g->in_col, icol.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !itv.empty())
        e = hipMemcpyAsync(g->in_task_v, itv.data(), sizeof(int32_t) * itv.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !ite.empty())
        e = hipMemcpyAsync(g->in_task_e0, ite.data(), sizeof(int64_t) * ite.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->in_task_start, its.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = imx::launch_thresholds(p_dev, g->W, m, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cleanup(IM_EDEVICE, std::string("graph upload: ") + hipGetErrorString(e));
    (void)hipFree(p_dev);
    p_dev = nullptr;
    *out = g;
    return IM_OK;
}

im_status im_graph_info(const im_graph* g, int64_t* n, int64_t* m)
{
    if (!g) return fail(IM_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    return IM_OK;
}

void im_graph_free(im_graph* g)
{
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    g->arena.release();
    delete g;
}

im_status im_sketch_build(const im_graph* g, int32_t J, uint64_t seed, void* stream, im_sketch** out)
{
    if (!out) return fail(IM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(IM_EINVAL, "graph is NULL");
    if (J < 64 || J > imx::kMaxJ || J % 64 != 0) return fail(IM_EINVAL, "J must be a multiple of 64 in [64, 4096]");
    const int64_t n = g->n;
    const size_t nJ = (size_t)n * (size_t)J;
    const size_t bm_words = (size_t)((n + 31) / 32);
    const size_t nt = (size_t)std::max<int64_t>(g->ntasks, 1), nit = (size_t)std::max<int64_t>(g->n_in_tasks, 1);
    size_t need = nJ + (size_t)n * (4 + 8 + 1 + 4 * 3) + bm_words * 12 + nt * 16 + nit * 4 + (1u << 20);
    size_t free_b = 0, total_b = 0;
    IMX_HIP(hipMemGetInfo(&free_b, &total_b));
    if (need + (64u << 20) > free_b) return fail(IM_ENOMEM, "sketch does not fit in device memory");

    im_sketch* s = new im_sketch();
    s->g = g;
    s->stream = static_cast<hipStream_t>(stream);
    s->J = J;
    s->seed = seed;
    auto bad = [&](im_status stc, const std::string& msg) {
        delete s;
        return fail(stc, msg);
    };
    Arena& A = s->arena;
    if (A.alloc(&s->M, nJ) || A.alloc(&s->X, (size_t)J + imx::kBuckets + 1) || A.alloc(&s->Ju, n) || A.alloc(&s->Hu, n) ||
        A.alloc(&s->sw.chg[0], bm_words) || A.alloc(&s->sw.chg[1], bm_words) || A.alloc(&s->sw.act_bm, bm_words) ||
        A.alloc(&s->sw.act_tasks[0], nt) || A.alloc(&s->sw.act_tasks[1], nt) || A.alloc(&s->sw.act_count, 4) ||
        A.alloc(&s->sw.chg_list, nit) || A.alloc(&s->sw.chg_count, 4) || A.alloc(&s->sw.rows_changed, 4) || A.alloc(&s->sw.dense, 4) ||
        A.alloc(&s->is_seed, n) || A.alloc(&s->best, 1) || A.alloc(&s->casc.q[0], nt) || A.alloc(&s->casc.q[1], nt) ||
        A.alloc(&s->casc.qsize, 4) || A.alloc(&s->casc.stamp, n) || A.alloc(&s->casc.touched, n) ||
        A.alloc(&s->casc.ntouched, 1) || A.alloc(&s->casc.touch_stamp, n) || A.alloc(&s->casc.T, 1) ||
        A.alloc(&s->am.pJ, imx::kArgmaxBlocks) || A.alloc(&s->am.pH, imx::kArgmaxBlocks) ||
        A.alloc(&s->am.pid, imx::kArgmaxBlocks))
        return bad(IM_ENOMEM, "device allocation failed");
    if (hipHostMalloc(reinterpret_cast<void**>(&s->h_ctr), sizeof(unsigned long long) * 4, 0) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_qs), sizeof(uint32_t) * 4, 0) != hipSuccess)
        return bad(IM_ENOMEM, "pinned host allocation failed");
    for (auto& e : s->ev)
        if (hipEventCreate(&e) != hipSuccess) return bad(IM_EDEVICE, "hipEventCreate failed");
    for (auto& e : s->evk)
        if (hipEventCreate(&e) != hipSuccess) return bad(IM_EDEVICE, "hipEventCreate failed");
    s->profiling = g_profiling.load();
    if (s->profiling >= 2 && A.alloc(&s->pc, 1)) return bad(IM_ENOMEM, "device allocation failed");

    hipStream_t st = s->stream;
    hipError_t e = hipMemsetAsync(s->is_seed, 0, n, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->casc.stamp, 0, sizeof(uint32_t) * n, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->casc.touch_stamp, 0, sizeof(uint32_t) * n, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->casc.T, 0, sizeof(unsigned long long), st);
    if (e == hipSuccess) e = hipEventRecord(s->ev[0], st);
    if (e == hipSuccess) e = imx::launch_sim_values(seed, J, s->X, st);
    if (e != hipSuccess) return bad(IM_EDEVICE, std::string("sketch init: ") + hipGetErrorString(e));
    int32_t sw = 0;
    if (im_status r = run_build(s, true, &sw)) {
        std::string msg = g_err;
        return bad(r, msg);
    }
    if (hipEventRecord(s->ev[1], st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return bad(IM_EDEVICE, "sketch build sync failed");
    s->st.build_sweeps = sw;
    s->st.build_ms = elapsed(s->ev[0], s->ev[1]);
    *out = s;
    return IM_OK;
}

im_status im_select_seeds(im_sketch* s, int32_t K, int32_t* seeds_host, double* spread_out, double* est_host,
                          uint64_t* T_host, im_stats* stats_out)
{
    if (!s) return fail(IM_EINVAL, "sketch is NULL");
    if (s->selected) return fail(IM_ESTATE, "seeds were already selected on this sketch; build a new one");
    const im_graph* g = s->g;
    if (K < 1 || K > g->n) return fail(IM_EINVAL, "K must be in [1, n]");
    if (!seeds_host) return fail(IM_EINVAL, "seeds output is NULL");
    hipStream_t st = s->stream;

    int32_t* seeds_dev = nullptr;
    uint32_t* pickJ = nullptr;
    unsigned long long* pickH = nullptr;
    Arena tmp;
    if (tmp.alloc(&seeds_dev, K) || tmp.alloc(&pickJ, K) || tmp.alloc(&pickH, K))
        return tmp.release(), fail(IM_ENOMEM, "device allocation failed");
    struct Guard {
        Arena& a;
        ~Guard() { a.release(); }
    } guard{tmp};

    s->selected = true;
    const imx::GraphDev gd = g->dev();
    std::vector<uint64_t> Tk(K);
    uint64_t T_old = 0;
    float casc_ms = 0.f;
    hipEvent_t e0, e1, c0, c1;
    IMX_HIP(hipEventCreate(&e0));
    IMX_HIP(hipEventCreate(&e1));
    IMX_HIP(hipEventCreate(&c0));
    IMX_HIP(hipEventCreate(&c1));
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard()
        {
            for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
        }
    };
    hipEvent_t evs[4] = {e0, e1, c0, c1};
    EvGuard eg{evs};
    IMX_HIP(hipEventRecord(e0, st));
    for (int32_t k = 0; k < K; ++k) {
        IMX_HIP(imx::launch_argmax(s->Ju, s->Hu, s->is_seed, g->n, s->am, s->best, st));
        IMX_HIP(hipEventRecord(c0, st));
        const uint32_t cid = ++s->cascade_id;
        const uint32_t base = s->level_base;
        IMX_HIP(imx::launch_cascade_seed(gd, s->best, k, s->M, s->J, s->is_seed, seeds_dev, pickJ, pickH, s->Ju,
                                         s->Hu, s->casc, cid, base + 1, st));
        int t = 1;
        for (;;) {
            for (int b = 0; b < kLevelBatch; ++b, ++t)
                IMX_HIP(imx::launch_cascade_level(gd, s->X, s->J, s->M, s->casc, t, base + (uint32_t)t + 1, cid, st));
            IMX_HIP(hipMemcpyAsync(s->h_qs, s->casc.qsize, sizeof(uint32_t) * 4, hipMemcpyDeviceToHost, st));
            IMX_HIP(hipStreamSynchronize(st));
            if (s->h_qs[t & 3] == 0) break;
            if (t > g->n + 8) return fail(IM_EDEVICE, "cascade did not terminate");
        }
        s->level_base = base + (uint32_t)t + 2;
        s->st.cascade_levels += t - 1;
        IMX_HIP(imx::launch_cascade_finalize(s->M, s->J, s->Ju, s->Hu, s->casc, st));
        IMX_HIP(hipEventRecord(c1, st));
        uint64_t T = 0;
        IMX_HIP(hipMemcpyAsync(s->h_ctr, s->casc.T, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        IMX_HIP(hipStreamSynchronize(st));
        T = s->h_ctr[0];
        casc_ms += elapsed(c0, c1);
        Tk[k] = T;
        if (k + 1 < K && 100 * (T - T_old) > T) {
            int32_t sw = 0;
            if (im_status r = run_build(s, false, &sw)) return r;
            ++s->st.rebuilds;
            T_old = T;
        }
    }
    IMX_HIP(hipEventRecord(e1, st));
    std::vector<uint32_t> hJ(K);
    std::vector<unsigned long long> hH(K);
    IMX_HIP(hipMemcpyAsync(seeds_host, seeds_dev, sizeof(int32_t) * K, hipMemcpyDeviceToHost, st));
    IMX_HIP(hipMemcpyAsync(hJ.data(), pickJ, sizeof(uint32_t) * K, hipMemcpyDeviceToHost, st));
    IMX_HIP(hipMemcpyAsync(hH.data(), pickH, sizeof(unsigned long long) * K, hipMemcpyDeviceToHost, st));
    IMX_HIP(hipStreamSynchronize(st));
    for (int32_t k = 0; k < K; ++k)
        if (seeds_host[k] < 0) return fail(IM_EDEVICE, "argmax found no candidate");
    s->st.select_ms = elapsed(e0, e1);
    s->st.cascade_ms = casc_ms;

    if (est_host) {
        const int J = s->J;
        const double alpha = (J == 16) ? 0.673 : (J == 32) ? 0.697 : (J == 64) ? 0.709 : 0.7213 / (1.0 + 1.079 / (double)J);
        const volatile double scale = alpha * 8589934592.0;
        for (int32_t k = 0; k < K; ++k) {
            if (hJ[k] == 0) {
                est_host[k] = 0.0;
                continue;
            }
            const volatile double num = (double)((uint64_t)hJ[k] * hJ[k]);
            const volatile double den = (double)J * (double)hH[k];
            const volatile double q = num / den;
            est_host[k] = scale * q;
        }
    }
    if (T_host)
        for (int32_t k = 0; k < K; ++k) T_host[k] = Tk[k];
    if (spread_out) *spread_out = (double)Tk[K - 1] / (double)s->J;
    if (stats_out) *stats_out = s->st;
    return IM_OK;
}

im_status im_sketch_registers(const im_sketch* s, uint8_t* regs_host)
{
    if (!s || !regs_host) return fail(IM_EINVAL, "NULL argument");
    IMX_HIP(hipMemcpyAsync(regs_host, s->M, (size_t)s->g->n * (size_t)s->J, hipMemcpyDeviceToHost, s->stream));
    IMX_HIP(hipStreamSynchronize(s->stream));
    return IM_OK;
}

im_status im_sketch_register_rows(const im_sketch* s, const int32_t* rows_host, int32_t nrows, uint8_t* regs_host)
{
    if (!s || nrows < 0 || (nrows > 0 && (!rows_host || !regs_host))) return fail(IM_EINVAL, "NULL argument");
    for (int32_t i = 0; i < nrows; ++i)
        if (rows_host[i] < 0 || rows_host[i] >= s->g->n) return fail(IM_EINVAL, "row id out of range");
    const size_t J = (size_t)s->J;
    for (int32_t i = 0; i < nrows; ++i)
        IMX_HIP(hipMemcpyAsync(regs_host + (size_t)i * J, s->M + (size_t)rows_host[i] * J, J, hipMemcpyDeviceToHost,
                               s->stream));
    IMX_HIP(hipStreamSynchronize(s->stream));
    return IM_OK;
}

im_status im_sketch_estimates(const im_sketch* s, uint32_t* Ju_host, uint64_t* Hu_host)
{
    if (!s) return fail(IM_EINVAL, "sketch is NULL");
    const int64_t n = s->g->n;
    if (Ju_host) IMX_HIP(hipMemcpyAsync(Ju_host, s->Ju, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s->stream));
    if (Hu_host) IMX_HIP(hipMemcpyAsync(Hu_host, s->Hu, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s->stream));
    IMX_HIP(hipStreamSynchronize(s->stream));
    return IM_OK;
}

im_status im_sketch_stats(const im_sketch* s, im_stats* out)
{
    if (!s || !out) return fail(IM_EINVAL, "NULL argument");
    *out = s->st;
    return IM_OK;
}

im_status im_sketch_sim_values(const im_sketch* s, uint32_t* X_host)
{
    if (!s || !X_host) return fail(IM_EINVAL, "NULL argument");
    IMX_HIP(hipMemcpyAsync(X_host, s->X, sizeof(uint32_t) * s->J, hipMemcpyDeviceToHost, s->stream));
    IMX_HIP(hipStreamSynchronize(s->stream));
    return IM_OK;
}

void im_sketch_free(im_sketch* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    delete s;
}

}  // extern "C"
