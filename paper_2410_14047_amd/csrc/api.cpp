// C-ABI host layer of libimx.so: errors, version, profiling switch and graph
// loading (validation, work decomposition, reverse graph, upload).  Sketches,
// engines and the batch entry point live in engine.cpp; every step of the
// method runs in the kernels of kernels.hip.
#include "handles.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;
std::atomic<int> g_profiling{0};

int default_split()
{
    const char* s = std::getenv("IMX_SPLIT");
    int v = s ? std::atoi(s) : 128;
    return (v >= 16 && v < (1 << 30)) ? v : 128;
}

im_status check_device()
{
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || cnt < 1) {
        g_err = "no HIP device available";
        return IM_EDEVICE;
    }
    return IM_OK;
}

}  // namespace

namespace imx {

im_status set_error(im_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

int profiling_level() { return g_profiling.load(); }

namespace {
std::mutex g_alloc_mutex;
DeviceAllocator g_alloc;
}  // namespace

DeviceAllocator current_allocator()
{
    std::lock_guard<std::mutex> lock(g_alloc_mutex);
    return g_alloc;
}

hipError_t device_alloc(size_t bytes, DeviceBlock* out)
{
    out->from = current_allocator();
    out->ptr = nullptr;
    if (out->from.alloc) {
        out->ptr = out->from.alloc(bytes, out->from.ctx);
        // blocks serve 16-byte vector loads
        if (out->ptr && (reinterpret_cast<uintptr_t>(out->ptr) & 15u)) {
            out->from.free_(out->ptr, out->from.ctx);
            out->ptr = nullptr;
        }
        return out->ptr ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(&out->ptr, bytes);
}

void device_free(const DeviceBlock& b)
{
    if (!b.ptr) return;
    if (b.from.free_)
        b.from.free_(b.ptr, b.from.ctx);
    else
        (void)hipFree(b.ptr);
}

}  // namespace imx

using imx::set_error;

extern "C" {

const char* im_last_error(void) { return g_err.c_str(); }

im_status im_version(int32_t* major, int32_t* minor)
{
    if (major) *major = 0;
    if (minor) *minor = 1;
    return IM_OK;
}

im_status im_set_allocator(im_alloc_fn alloc, im_free_fn free_, void* ctx)
{
    if ((alloc == nullptr) != (free_ == nullptr)) return set_error(IM_EINVAL, "set both hooks or neither");
    std::lock_guard<std::mutex> lock(imx::g_alloc_mutex);
    imx::g_alloc = imx::DeviceAllocator{alloc, free_, alloc ? ctx : nullptr};
    return IM_OK;
}

im_status im_set_profiling(int32_t level)
{
    if (level < 0 || level > 2) return set_error(IM_EINVAL, "profiling level must be 0, 1 or 2");
    g_profiling.store(level);
    return IM_OK;
}

im_status im_graph_load(int64_t n, int64_t m, const int64_t* rowptr_host, const int32_t* col_host,
                        const float* p_host, void* stream, im_graph** out)
{
    if (!out) return set_error(IM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= (int64_t(1) << 31)) return set_error(IM_EINVAL, "n must be in [1, 2^31)");
    if (m < 0 || m >= (int64_t(1) << 40)) return set_error(IM_EINVAL, "m must be in [0, 2^40)");
    if (!rowptr_host || (m > 0 && (!col_host || !p_host))) return set_error(IM_EINVAL, "NULL array");
    if (rowptr_host[0] != 0) return set_error(IM_EINVAL, "rowptr[0] != 0");
    if (rowptr_host[n] != m) return set_error(IM_EINVAL, "rowptr[n] != m");
    for (int64_t u = 0; u < n; ++u) {
        const int64_t b = rowptr_host[u], e = rowptr_host[u + 1];
        if (e < b) return set_error(IM_EINVAL, "rowptr decreases at vertex " + std::to_string(u));
        for (int64_t i = b; i < e; ++i) {
            const int32_t v = col_host[i];
            if (v < 0 || v >= n) return set_error(IM_EINVAL, "col out of range at arc " + std::to_string(i));
            if (i > b && v <= col_host[i - 1])
                return set_error(IM_EINVAL, "col not strictly increasing within row at arc " + std::to_string(i));
            const float p = p_host[i];
            if (!(p >= 0.0f && p <= 1.0f)) return set_error(IM_EINVAL, "p outside [0,1] at arc " + std::to_string(i));
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
    if ((int64_t)tu.size() >= (int64_t(1) << 31)) return set_error(IM_EINVAL, "too many propagation tasks");
    // Order of a sweep that visits every task: heavy classes first (arc
    // counts >= 64, >= 16, >= 4, the rest; task id order within a class), so
    // the packs dealt to workgroups in turn carry similar work and the light
    // ones fill in at the end, while most tasks keep the id order that makes
    // their rows and arcs nearly sequential.  (A full sort by arc count
    // balanced as well but slowed the bandwidth-bound sweeps of large
    // uniform-probability graphs, where rows read in id order stream.)
    std::vector<int32_t> dord(tu.size());
    {
        auto cls = [&](size_t t) {
            const uint32_t l = tl[t] & 0x7fffffffu;
            return l >= 64 ? 0 : l >= 16 ? 1 : l >= 4 ? 2 : 3;
        };
        int64_t cnt[5] = {0, 0, 0, 0, 0};
        for (size_t t = 0; t < tl.size(); ++t) ++cnt[cls(t) + 1];
        for (int i = 1; i < 5; ++i) cnt[i] += cnt[i - 1];
        for (size_t t = 0; t < tl.size(); ++t) dord[(size_t)cnt[cls(t)]++] = (int32_t)t;
    }
    std::vector<int32_t> du(dord.size());
    std::vector<int64_t> de(dord.size());
    std::vector<uint32_t> dl(dord.size());
    for (size_t i = 0; i < dord.size(); ++i) {
        du[i] = tu[(size_t)dord[i]];
        de[i] = te[(size_t)dord[i]];
        dl[i] = tl[(size_t)dord[i]];
    }
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

    size_t need = sizeof(int64_t) * (n + 1) * 2 + (size_t)m * 16 + tu.size() * 32 + itv.size() * 12 + (size_t)n * 8;
    size_t free_b = 0, total_b = 0;
    IMX_HIP(hipMemGetInfo(&free_b, &total_b));
    if (need + (64u << 20) > free_b) return set_error(IM_ENOMEM, "graph does not fit in device memory");

    im_graph* g = new im_graph();
    g->stream = static_cast<hipStream_t>(stream);
    g->n = n;
    g->m = m;
    g->split = split;
    g->ntasks = (int64_t)tu.size();
    g->in_split = in_split;
    g->n_in_tasks = (int64_t)itv.size();
    for (int64_t v = 0; v < n; ++v) {
        g->max_out_deg = std::max<int64_t>(g->max_out_deg, rowptr_host[v + 1] - rowptr_host[v]);
        g->max_in_deg = std::max<int64_t>(g->max_in_deg, irp[v + 1] - irp[v]);
    }
    float* p_dev = nullptr;
    imx::Arena tmp;  // probabilities, freed after the thresholds are computed
    auto cleanup = [&](im_status st, const std::string& msg) {
        tmp.release();
        g->arena.release();
        delete g;
        return set_error(st, msg);
    };
    imx::Arena& A = g->arena;
    if (A.alloc(&g->rowptr, n + 1) || A.alloc(&g->col, m) || A.alloc(&g->W, m) || A.alloc(&g->task_u, tu.size()) ||
        A.alloc(&g->task_e0, te.size()) || A.alloc(&g->task_len, tl.size()) || A.alloc(&g->task_start, n + 1) || A.alloc(&g->in_rowptr, n + 1) ||
        A.alloc(&g->in_col, m) || A.alloc(&g->in_task_v, itv.size()) || A.alloc(&g->in_task_e0, ite.size()) ||
        A.alloc(&g->in_task_start, n + 1) || A.alloc(&g->dense_u, du.size()) || A.alloc(&g->dense_e0, de.size()) ||
        A.alloc(&g->dense_len, dl.size()) || tmp.alloc(&p_dev, (size_t)m))
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
    if (e == hipSuccess && !du.empty())
        e = hipMemcpyAsync(g->dense_u, du.data(), sizeof(int32_t) * du.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !de.empty())
        e = hipMemcpyAsync(g->dense_e0, de.data(), sizeof(int64_t) * de.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !dl.empty())
        e = hipMemcpyAsync(g->dense_len, dl.data(), sizeof(uint32_t) * dl.size(), hipMemcpyHostToDevice, st);
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
    tmp.release();
    p_dev = nullptr;
    *out = g;
    return IM_OK;
}

im_status im_graph_info(const im_graph* g, int64_t* n, int64_t* m)
{
    if (!g) return set_error(IM_EINVAL, "graph is NULL");
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

}  // extern "C"
