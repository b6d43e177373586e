// Access-rate probe of the device memory system (a measurement aid for the
// propagation kernel's roofline, not part of the method).  It times, on a
// buffer far larger than every cache:
//   - gathers of G bytes (G = 16, 64, 128, 256, 1024) from uniformly random
//     G-aligned (16-byte gathers: 64-byte-aligned) positions, each gather
//     served by G/16 lanes with one 16-byte load each;
//   - a streaming read and a streaming copy.
// Every index is reduced modulo the number of positions, so all accesses stay
// in bounds.  Built as its own library (libimx_probe.so); bench.py calls it.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t splitmix(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// LPS lanes serve one gather of 16*LPS bytes; positions are STRIDE uint4 apart.
template <int LPS, int STRIDE>
__global__ void k_gather(const uint4* __restrict__ buf, uint64_t npos, int iters, uint64_t seed, uint32_t* out)
{
    const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t grp = tid / LPS;
    const int sub = (int)(tid % LPS);
    uint32_t acc = 0;
#pragma unroll 8
    for (int i = 0; i < iters; ++i) {
        const uint64_t p = splitmix(seed ^ (grp * 0x100000001b3ull + (uint64_t)i)) % npos;
        const uint4 v = buf[p * STRIDE + sub];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    out[tid] = acc;
}

__global__ void k_stream_read(const uint4* __restrict__ a, uint64_t n, uint32_t* out)
{
    uint32_t acc = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 v = a[i];
        acc ^= v.x ^ v.w;
    }
    out[blockIdx.x * (uint64_t)blockDim.x + threadIdx.x] = acc;
}

__global__ void k_stream_copy(const uint4* __restrict__ a, uint4* __restrict__ b, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

}  // namespace

extern "C" {

// Runs the probe on a buffer of `buffer_bytes` (a multiple of 1 MiB, at least
// 64 MiB; the copy uses a second buffer of a quarter of it).  Writes 7
// figures to out: gathers per second for G = 16, 64, 128, 256, 1024, then
// streaming read bytes/s and streaming copy bytes/s (read + write).  Returns
// 0 on success, else the HIP error code.  Allocates and frees its buffers.
int imx_probe_rates(uint64_t buffer_bytes, double* out)
{
    if (!out || buffer_bytes < (64ull << 20) || buffer_bytes % (1ull << 20)) return (int)hipErrorInvalidValue;
    uint4* buf = nullptr;
    uint4* dst = nullptr;
    uint32_t* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int blocks = 2048, threads = 256, iters = 64;
    const uint64_t nthreads = (uint64_t)blocks * threads;
    const uint64_t n16 = buffer_bytes / 16, ncopy = n16 / 4;
    hipError_t err = hipMalloc(&buf, buffer_bytes);
    if (err == hipSuccess) err = hipMalloc(&dst, ncopy * 16);
    if (err == hipSuccess) err = hipMalloc(&sink, nthreads * 4);
    if (err == hipSuccess) err = hipMemset(buf, 1, buffer_bytes);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    auto timed = [&](auto launch, double work, double* res) {
        if (err != hipSuccess) return;
        launch();
        err = hipDeviceSynchronize();
        if (err != hipSuccess) return;
        const int reps = 5;
        err = hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps; ++r) launch();
        if (err == hipSuccess) err = hipEventRecord(e1, nullptr);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess) err = hipGetLastError();
        *res = work / (ms * 1e-3 / reps);
    };
    timed([&] { hipLaunchKernelGGL((k_gather<1, 4>), dim3(blocks), dim3(threads), 0, nullptr, buf, n16 / 4, iters, 7ull, sink); },
          (double)nthreads * iters, &out[0]);
    timed([&] { hipLaunchKernelGGL((k_gather<4, 4>), dim3(blocks), dim3(threads), 0, nullptr, buf, n16 / 4, iters, 7ull, sink); },
          (double)nthreads / 4 * iters, &out[1]);
    timed([&] { hipLaunchKernelGGL((k_gather<8, 8>), dim3(blocks), dim3(threads), 0, nullptr, buf, n16 / 8, iters, 7ull, sink); },
          (double)nthreads / 8 * iters, &out[2]);
    timed([&] { hipLaunchKernelGGL((k_gather<16, 16>), dim3(blocks), dim3(threads), 0, nullptr, buf, n16 / 16, iters, 7ull, sink); },
          (double)nthreads / 16 * iters, &out[3]);
    timed([&] { hipLaunchKernelGGL((k_gather<64, 64>), dim3(blocks), dim3(threads), 0, nullptr, buf, n16 / 64, iters, 7ull, sink); },
          (double)nthreads / 64 * iters, &out[4]);
    timed([&] { hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(threads), 0, nullptr, buf, n16, sink); },
          (double)buffer_bytes, &out[5]);
    timed([&] { hipLaunchKernelGGL(k_stream_copy, dim3(256 * 16), dim3(256), 0, nullptr, buf, dst, ncopy); },
          2.0 * (double)ncopy * 16, &out[6]);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    if (dst) (void)hipFree(dst);
    if (buf) (void)hipFree(buf);
    return (int)err;
}

}  // extern "C"
