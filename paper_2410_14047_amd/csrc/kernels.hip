// HIP kernels for gfx950 (MI355X): fused hash sampling, register fill,
// pull-based propagation, estimate, argmax and the union-frontier cascade.
//
// Register layout: M is uint8[n][J], vertex-major, registers of a row in
// increasing (sorted-X) simulation order.  Uncovered registers hold
// rank values 1..33; covered registers hold 0.  During a cascade, registers
// covered at frontier level t temporarily hold the marker 64 + (t mod 64).
#include "imx_internal.h"

#include <hip/hip_runtime.h>

namespace imx {

// ---------------------------------------------------------------------------
// MurmurHash3_x86_32 pieces (published algorithm by A. Appleby).

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

__device__ __forceinline__ uint32_t mix_block(uint32_t h, uint32_t k)
{
    k *= 0xcc9e2d51u;
    k = rotl32(k, 15);
    k *= 0x1b873593u;
    h ^= k;
    h = rotl32(h, 13);
    return h * 5u + 0xe6546b64u;
}

__device__ __forceinline__ uint32_t finish(uint32_t h, uint32_t len)
{
    h ^= len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Eq. 1: 31-bit hash of arc (u, v), key = u || v (little-endian words), seed 0.
__device__ __forceinline__ uint32_t arc_hash(uint32_t u, uint32_t v)
{
    return finish(mix_block(mix_block(0u, u), v), 8u) & 0x7fffffffu;
}

// Per-row prefix of the register hash: key = seed_lo || seed_hi || u || j, seed 1.
__device__ __forceinline__ uint32_t rank_prefix(uint64_t seed, uint32_t u)
{
    return mix_block(mix_block(mix_block(1u, (uint32_t)seed), (uint32_t)(seed >> 32)), u);
}

// Eq. 3 with the HyperLogLog offset: leading zeros of the j-th hash, plus one.
__device__ __forceinline__ uint32_t rank_of(uint32_t prefix, uint32_t j)
{
    uint32_t g = finish(mix_block(prefix, j), 16u);
    return (g == 0u ? 32u : (uint32_t)__builtin_clz(g)) + 1u;
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64).

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Orders this wave's LDS traffic: everything written before is visible to
// every lane of the wave after it.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_incl_scan(int x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// First index i in sorted X[0..J) with X[i] >= key.
__device__ __forceinline__ int lower_bound_lds(const uint32_t* X, int J, uint32_t key)
{
    int lo = 0, len = J;
    while (len > 0) {
        int half = len >> 1;
        if (X[lo + half] < key) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// Candidate simulations of an arc with hash h and threshold W: since X is
// sorted and (X xor h) < W <= 2^b forces X >> b == h >> b, every live
// simulation lies in one contiguous index range [lo, hi) of X.
__device__ __forceinline__ void candidate_range(const uint32_t* X, int J, uint32_t h, uint32_t W, int& lo, int& hi)
{
    if (W == 0u) {
        lo = hi = 0;
    } else if (W >= 0x80000000u) {
        lo = 0;
        hi = J;
    } else {
        int b = (W == 1u) ? 0 : 32 - __builtin_clz(W - 1u);
        uint32_t base = (h >> b) << b;
        lo = lower_bound_lds(X, J, base);
        hi = lower_bound_lds(X, J, base + (1u << b));
    }
}

// Largest k in [0,64) with start[k] <= idx (start non-decreasing, start[0] = 0).
__device__ __forceinline__ int owner_of(const int* start, int idx)
{
    int k = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (start[k + step] <= idx) k += step;
    return k;
}

__device__ __forceinline__ uint32_t bytemax4(uint32_t a, uint32_t b)
{
    uint32_t r = 0;
#pragma unroll
    for (int s = 0; s < 32; s += 8) {
        uint32_t x = (a >> s) & 0xffu, y = (b >> s) & 0xffu;
        r |= (x > y ? x : y) << s;
    }
    return r;
}

// Wave-aggregated append of `v` (lanes with push) to queue Q with counter ctr.
__device__ __forceinline__ void wave_append(bool push, int32_t v, int32_t* Q, uint32_t* ctr)
{
    const int lane = lane_id();
    unsigned long long bal = __ballot(push);
    if (bal == 0ull) return;
    int leader = __ffsll((long long)bal) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(ctr, (uint32_t)__popcll(bal));
    base = __shfl(base, leader, 64);
    if (push) {
        uint32_t off = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        Q[base + off] = v;
    }
}

// ---------------------------------------------------------------------------
// a1: fixed-point thresholds W = min(2^31, floor(p * 2^31)).

__global__ void k_thresholds(const float* __restrict__ p, uint32_t* __restrict__ W, int64_t m)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        double w = (double)p[e] * 2147483648.0;
        uint32_t t = (w >= 2147483648.0) ? 0x80000000u : (w <= 0.0 ? 0u : (uint32_t)w);
        W[e] = t;
    }
}

hipError_t launch_thresholds(const float* p, uint32_t* W, int64_t m, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_thresholds, dim3((unsigned)blocks), dim3(256), 0, st, p, W, m);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a2: simulation values X: top 31 bits of SplitMix64 outputs 0..J-1, sorted
// ascending with a bitonic network in LDS (one workgroup).

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(1024) void k_sim_values(uint64_t seed, int J, uint32_t* __restrict__ X)
{
    __shared__ uint32_t s[kMaxJ];
    int P = 1;
    while (P < J) P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x)
        s[i] = (i < J) ? (uint32_t)(splitmix64_at(seed, (uint64_t)i) >> 33) : 0xffffffffu;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint32_t a = s[i], b = s[ixj];
                    bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        s[i] = b;
                        s[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < J; i += blockDim.x) X[i] = s[i];
}

hipError_t launch_sim_values(uint64_t seed, int J, uint32_t* X, hipStream_t st)
{
    hipLaunchKernelGGL(k_sim_values, dim3(1), dim3(1024), 0, st, seed, J, X);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a3: Fill-Sketches (Alg. 1).  One thread per 4 registers.  On a rebuild,
// covered registers (0) stay 0.

__global__ void k_fill(uint8_t* __restrict__ M, int64_t n, int J, uint64_t seed, int first)
{
    const int64_t words_per_row = J / 4;
    const int64_t total = n * words_per_row;
    uint32_t* M32 = reinterpret_cast<uint32_t*>(M);
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < total; d += (int64_t)gridDim.x * blockDim.x) {
        uint32_t u = (uint32_t)(d / words_per_row);
        uint32_t j0 = (uint32_t)(d - (int64_t)u * words_per_row) * 4u;
        uint32_t pre = rank_prefix(seed, u);
        uint32_t old = first ? 0xffffffffu : M32[d];
        uint32_t out = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint32_t r = ((old >> (8 * b)) & 0xffu) ? rank_of(pre, j0 + b) : 0u;
            out |= r << (8 * b);
        }
        M32[d] = out;
    }
}

hipError_t launch_fill(uint8_t* M, int64_t n, int J, uint64_t seed, bool first, hipStream_t st)
{
    int64_t total = n * (J / 4);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 262144) blocks = 262144;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, M, n, J, seed, first ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a4: one propagation sweep (Alg. 2, pull-based, in place).
//
// One wave per task (a vertex u, or a run of at most `split` of its out-arcs).
// Lane-per-arc phase: arc hash, threshold, candidate range from sorted X, and
// the frontier filter (only arcs whose head changed in the previous sweep).
// Flattened phase: the (arc, candidate simulation) pairs of 64 arcs are dealt
// to lanes; each lane tests liveness (Eq. 2) and max-merges the head's
// register into u's row, kept as one 32-bit word per simulation in LDS.
// Finally the row is packed to bytes; changed words are stored (split rows
// merge with a byte-max compare-and-swap) and u is flagged in chg_next.

struct PropArgs {
    GraphDev g;
    const uint32_t* X;
    int J;
    uint8_t* M;
    const uint32_t* chg_prev;
    uint32_t* chg_next;
    unsigned long long* changed;
};

constexpr int kEdgeBufWords = 5 * 64;

template <int DPL>
__global__ __launch_bounds__(kWG) void k_propagate(PropArgs a)
{
    extern __shared__ uint32_t smem[];
    const int J = a.J;
    const int Jw = J >> 2;  // 32-bit words per row
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = lane_id();
    uint32_t* sX = smem;
    uint32_t* row = smem + J + wave * (J + kEdgeBufWords);
    int* ev = reinterpret_cast<int*>(row + J);
    uint32_t* eh = row + J + 64;
    uint32_t* eW = row + J + 128;
    int* elo = reinterpret_cast<int*>(row + J + 192);
    int* est = reinterpret_cast<int*>(row + J + 256);

    for (int i = threadIdx.x; i < J; i += kWG) sX[i] = a.X[i];
    __syncthreads();

    const GraphDev& g = a.g;
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t t = (int64_t)blockIdx.x * kWaves + wave; t < g.ntasks; t += nw) {
        const int32_t u = g.task_u[t];
        const int64_t rb = g.rowptr[u], re = g.rowptr[u + 1];
        const int64_t e0 = g.task_e0[t];
        const int64_t e1 = (e0 + g.split < re) ? e0 + g.split : re;
        const bool split = (re - rb) > (int64_t)g.split;
        uint8_t* Mu = a.M + (size_t)u * (size_t)J;
        uint32_t saved[DPL];
        bool init = false;

        for (int64_t cb = e0; cb < e1; cb += 64) {
            const int64_t e = cb + lane;
            int cnt = 0, lo = 0;
            int32_t v = 0;
            uint32_t h = 0, w = 0;
            if (e < e1) {
                v = g.col[e];
                if ((a.chg_prev[(uint32_t)v >> 5] >> (v & 31)) & 1u) {
                    w = g.W[e];
                    h = arc_hash((uint32_t)u, (uint32_t)v);
                    int hi;
                    candidate_range(sX, J, h, w, lo, hi);
                    cnt = hi - lo;
                }
            }
            const int incl = wave_incl_scan(cnt);
            const int total = __shfl(incl, 63, 64);
            if (total == 0) continue;
            if (!init) {
#pragma unroll
                for (int i = 0; i < DPL; ++i) {
                    const int idx = lane + 64 * i;
                    if (idx < Jw) {
                        uint32_t d = reinterpret_cast<const uint32_t*>(Mu)[idx];
                        saved[i] = d;
                        uint4 w4;
                        w4.x = d & 0xffu;
                        w4.y = (d >> 8) & 0xffu;
                        w4.z = (d >> 16) & 0xffu;
                        w4.w = d >> 24;
                        *reinterpret_cast<uint4*>(&row[4 * idx]) = w4;
                    }
                }
                init = true;
            }
            ev[lane] = v;
            eh[lane] = h;
            eW[lane] = w;
            elo[lane] = lo;
            est[lane] = incl - cnt;
            wave_lds_sync();
            for (int r = 0; r < total; r += 64) {
                const int idx = r + lane;
                if (idx < total) {
                    const int k = owner_of(est, idx);
                    const int j = elo[k] + (idx - est[k]);
                    if ((sX[j] ^ eh[k]) < eW[k]) {
                        uint32_t val = a.M[(size_t)ev[k] * (size_t)J + (size_t)j];
                        atomicMax(&row[j], val);
                    }
                }
            }
            wave_lds_sync();
        }

        if (init) {
            bool changed = false;
#pragma unroll
            for (int i = 0; i < DPL; ++i) {
                const int idx = lane + 64 * i;
                if (idx < Jw) {
                    uint4 w4 = *reinterpret_cast<const uint4*>(&row[4 * idx]);
                    uint32_t nwd = w4.x | (w4.y << 8) | (w4.z << 16) | (w4.w << 24);
                    if (nwd != saved[i]) {
                        uint32_t* addr = reinterpret_cast<uint32_t*>(Mu) + idx;
                        if (!split) {
                            *addr = nwd;
                            changed = true;
                        } else {
                            uint32_t cur = __hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            for (;;) {
                                uint32_t want = bytemax4(cur, nwd);
                                if (want == cur) break;
                                uint32_t prev = atomicCAS(addr, cur, want);
                                if (prev == cur) {
                                    changed = true;
                                    break;
                                }
                                cur = prev;
                            }
                        }
                    }
                }
            }
            const unsigned long long bal = __ballot(changed);
            if (bal != 0ull && lane == 0) {
                atomicOr(&a.chg_next[(uint32_t)u >> 5], 1u << (u & 31));
                atomicAdd(a.changed, 1ull);
            }
            wave_lds_sync();
        }
    }
}

template <int DPL>
static hipError_t launch_propagate_t(const PropArgs& a, hipStream_t st)
{
    static int grid = 0;
    const size_t lds = sizeof(uint32_t) * ((size_t)a.J + (size_t)kWaves * ((size_t)a.J + kEdgeBufWords));
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_propagate<DPL>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    int per_cu = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_propagate<DPL>, kWG, lds);
    if (err != hipSuccess) return err;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (per_cu < 1) per_cu = 1;
    grid = cus * per_cu;
    int64_t need = (a.g.ntasks + kWaves - 1) / kWaves;
    if (need < grid) grid = (int)(need > 0 ? need : 1);
    hipLaunchKernelGGL(k_propagate<DPL>, dim3(grid), dim3(kWG), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_propagate(const GraphDev& g, const uint32_t* X, int J, uint8_t* M, const uint32_t* chg_prev,
                            uint32_t* chg_next, unsigned long long* changed, hipStream_t st)
{
    PropArgs a{g, X, J, M, chg_prev, chg_next, changed};
    if (g.ntasks == 0) return hipSuccess;
    if (J <= 256) return launch_propagate_t<1>(a, st);
    if (J <= 512) return launch_propagate_t<2>(a, st);
    if (J <= 1024) return launch_propagate_t<4>(a, st);
    if (J <= 2048) return launch_propagate_t<8>(a, st);
    return launch_propagate_t<16>(a, st);
}

// ---------------------------------------------------------------------------
// a5: estimate terms per vertex (Eq. 7 harmonic form over uncovered registers):
// Ju = #registers != 0, Hu = sum of 2^(33 - M).  One wave per row.

__global__ __launch_bounds__(kWG) void k_estimate(const uint8_t* __restrict__ M, int64_t n, int J,
                                                   uint32_t* __restrict__ Ju, unsigned long long* __restrict__ Hu)
{
    const int lane = lane_id();
    const int Jw = J >> 2;
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t v = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); v < n; v += nw) {
        const uint32_t* row = reinterpret_cast<const uint32_t*>(M + (size_t)v * (size_t)J);
        uint32_t c = 0;
        unsigned long long h = 0;
        for (int idx = lane; idx < Jw; idx += 64) {
            uint32_t d = row[idx];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                uint32_t r = (d >> (8 * b)) & 0xffu;
                if (r) {
                    ++c;
                    h += 1ull << (33u - r);
                }
            }
        }
        c = wave_sum_u32(c);
        h = wave_sum_u64(h);
        if (lane == 0) {
            Ju[v] = c;
            Hu[v] = h;
        }
    }
}

hipError_t launch_estimate(const uint8_t* M, int64_t n, int J, uint32_t* Ju, unsigned long long* Hu, hipStream_t st)
{
    int64_t blocks = (n + kWaves - 1) / kWaves;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_estimate, dim3((unsigned)blocks), dim3(kWG), 0, st, M, n, J, Ju, Hu);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a6: argmax over non-seeds of J_u^2 / H_u, compared exactly with 128-bit
// cross products; value 0 when J_u = 0; ties go to the lowest id.  Any
// reduction order gives the same winner.

struct Cand {
    uint32_t J;
    unsigned long long H;
    int32_t id;
};

__device__ __forceinline__ bool better(const Cand& a, const Cand& b)
{
    if (a.id < 0) return false;
    if (b.id < 0) return true;
    if (a.J == 0u || b.J == 0u) {
        if (a.J == 0u && b.J == 0u) return a.id < b.id;
        return b.J == 0u;
    }
    const unsigned long long a2 = (unsigned long long)a.J * a.J, b2 = (unsigned long long)b.J * b.J;
    const unsigned long long lhi = __umul64hi(a2, b.H), llo = a2 * b.H;
    const unsigned long long rhi = __umul64hi(b2, a.H), rlo = b2 * a.H;
    if (lhi != rhi) return lhi > rhi;
    if (llo != rlo) return llo > rlo;
    return a.id < b.id;
}

__device__ void block_reduce_best(Cand& c)
{
    __shared__ uint32_t sJ[256];
    __shared__ unsigned long long sH[256];
    __shared__ int32_t sI[256];
    const int t = threadIdx.x;
    sJ[t] = c.J;
    sH[t] = c.H;
    sI[t] = c.id;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (t < s) {
            Cand o{sJ[t + s], sH[t + s], sI[t + s]};
            Cand m{sJ[t], sH[t], sI[t]};
            if (better(o, m)) {
                sJ[t] = o.J;
                sH[t] = o.H;
                sI[t] = o.id;
            }
        }
        __syncthreads();
    }
    c = Cand{sJ[0], sH[0], sI[0]};
}

__global__ __launch_bounds__(256) void k_argmax_partial(const uint32_t* __restrict__ Ju,
                                                         const unsigned long long* __restrict__ Hu,
                                                         const uint8_t* __restrict__ is_seed, int64_t n,
                                                         ArgmaxScratch s)
{
    Cand best{0u, 0ull, -1};
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (is_seed[v]) continue;
        Cand c{Ju[v], Hu[v], (int32_t)v};
        if (better(c, best)) best = c;
    }
    block_reduce_best(best);
    if (threadIdx.x == 0) {
        s.pJ[blockIdx.x] = best.J;
        s.pH[blockIdx.x] = best.H;
        s.pid[blockIdx.x] = best.id;
    }
}

__global__ __launch_bounds__(256) void k_argmax_final(ArgmaxScratch s, int nparts, int32_t* best_out)
{
    Cand best{0u, 0ull, -1};
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        Cand c{s.pJ[i], s.pH[i], s.pid[i]};
        if (better(c, best)) best = c;
    }
    block_reduce_best(best);
    if (threadIdx.x == 0) *best_out = best.id;
}

hipError_t launch_argmax(const uint32_t* Ju, const unsigned long long* Hu, const uint8_t* is_seed, int64_t n,
                         const ArgmaxScratch& s, int32_t* best, hipStream_t st)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > kArgmaxBlocks) blocks = kArgmaxBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_argmax_partial, dim3((unsigned)blocks), dim3(256), 0, st, Ju, Hu, is_seed, n, s);
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(256), 0, st, s, (int)blocks, best);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a7: covering cascade (Alg. 3), union-frontier BFS over all simulations.

__device__ __forceinline__ uint32_t marker(int t) { return 64u + ((uint32_t)t & 63u); }
__device__ __forceinline__ bool uncovered(uint32_t b) { return b >= 1u && b <= 33u; }

// Level 0: the pick s becomes a seed and is covered in every simulation where
// it is not yet covered; s forms frontier Q_1.
__global__ __launch_bounds__(64) void k_cascade_seed(const int32_t* __restrict__ best, int32_t k, uint8_t* M, int J,
                                                      uint8_t* is_seed, int32_t* seeds, uint32_t* pickJ,
                                                      unsigned long long* pickH, const uint32_t* Ju,
                                                      const unsigned long long* Hu, CascadeDev c,
                                                      uint32_t cascade_id, uint32_t level_id1)
{
    const int lane = lane_id();
    const int32_t s = *best;
    if (s < 0) {  // no candidate (cannot happen for K <= n); leave an empty cascade
        if (lane == 0) {
            seeds[k] = -1;
            c.qsize[0] = c.qsize[1] = c.qsize[2] = c.qsize[3] = 0;
            *c.ntouched = 0;
        }
        return;
    }
    uint32_t* row = reinterpret_cast<uint32_t*>(M + (size_t)s * (size_t)J);
    bool any = false;
    const uint32_t mk = marker(0);
    for (int idx = lane; idx < (J >> 2); idx += 64) {
        uint32_t d = row[idx], o = d;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint32_t r = (d >> (8 * b)) & 0xffu;
            if (uncovered(r)) d = (d & ~(0xffu << (8 * b))) | (mk << (8 * b));
        }
        if (d != o) {
            row[idx] = d;
            any = true;
        }
    }
    const unsigned long long bal = __ballot(any);
    if (lane == 0) {
        is_seed[s] = 1;
        seeds[k] = s;
        pickJ[k] = Ju[s];
        pickH[k] = Hu[s];
        c.qsize[0] = 0;
        c.qsize[2] = 0;
        c.qsize[3] = 0;
        c.qsize[1] = bal ? 1u : 0u;
        c.q[1][0] = s;
        c.stamp[s] = level_id1;
        c.touched[0] = s;
        *c.ntouched = 1;
        c.touch_stamp[s] = cascade_id;
    }
}

hipError_t launch_cascade_seed(const int32_t* best, int32_t k, uint8_t* M, int J, uint8_t* is_seed, int32_t* seeds,
                               uint32_t* pickJ, unsigned long long* pickH, const uint32_t* Ju,
                               const unsigned long long* Hu, const CascadeDev& c, uint32_t cascade_id,
                               uint32_t level_id1, hipStream_t st)
{
    hipLaunchKernelGGL(k_cascade_seed, dim3(1), dim3(64), 0, st, best, k, M, J, is_seed, seeds, pickJ, pickH, Ju, Hu,
                       c, cascade_id, level_id1);
    return hipGetLastError();
}

// Level t >= 1: expand every u in Q_t along its live arcs in the simulations
// where u was covered at level t-1; heads still uncovered there become covered
// (marker of level t) and join Q_{t+1}.  One wave per frontier vertex.
struct LevelArgs {
    GraphDev g;
    const uint32_t* X;
    int J;
    uint8_t* M;
    CascadeDev c;
    int t;
    uint32_t level_id;    // stamp of Q_{t+1}
    uint32_t cascade_id;
};

constexpr int kLevelBufWords = 6 * 64;

__global__ __launch_bounds__(kWG) void k_cascade_level(LevelArgs a)
{
    extern __shared__ uint32_t smem[];
    const int J = a.J;
    const int Jw = J >> 2;
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = lane_id();
    uint32_t* sX = smem;
    uint32_t* roww = smem + J + wave * (Jw + kLevelBufWords);
    const uint8_t* rowb = reinterpret_cast<const uint8_t*>(roww);
    int* ev = reinterpret_cast<int*>(roww + Jw);
    uint32_t* eh = roww + Jw + 64;
    uint32_t* eW = roww + Jw + 128;
    int* elo = reinterpret_cast<int*>(roww + Jw + 192);
    int* est = reinterpret_cast<int*>(roww + Jw + 256);
    uint32_t* efl = roww + Jw + 320;

    if (blockIdx.x == 0 && threadIdx.x == 0) a.c.qsize[(a.t + 2) & 3] = 0;
    for (int i = threadIdx.x; i < J; i += kWG) sX[i] = a.X[i];
    __syncthreads();

    const uint32_t qn = a.c.qsize[a.t & 3];
    const int32_t* Q = a.c.q[a.t & 1];
    int32_t* Qn = a.c.q[(a.t + 1) & 1];
    uint32_t* qn_ctr = &a.c.qsize[(a.t + 1) & 3];
    const uint8_t mk_prev = (uint8_t)marker(a.t - 1);
    const uint8_t mk_cur = (uint8_t)marker(a.t);
    const GraphDev& g = a.g;
    const int64_t nw = (int64_t)gridDim.x * kWaves;

    for (int64_t i = (int64_t)blockIdx.x * kWaves + wave; i < (int64_t)qn; i += nw) {
        const int32_t u = Q[i];
        const uint32_t* Mu = reinterpret_cast<const uint32_t*>(a.M + (size_t)u * (size_t)J);
        for (int idx = lane; idx < Jw; idx += 64) roww[idx] = Mu[idx];
        wave_lds_sync();
        const int64_t rb = g.rowptr[u], re = g.rowptr[u + 1];
        for (int64_t cb = rb; cb < re; cb += 64) {
            const int64_t e = cb + lane;
            int cnt = 0, lo = 0;
            int32_t v = 0;
            uint32_t h = 0, w = 0;
            if (e < re) {
                v = g.col[e];
                w = g.W[e];
                h = arc_hash((uint32_t)u, (uint32_t)v);
                int hi;
                candidate_range(sX, J, h, w, lo, hi);
                cnt = hi - lo;
            }
            const int incl = wave_incl_scan(cnt);
            const int total = __shfl(incl, 63, 64);
            if (total == 0) continue;
            ev[lane] = v;
            eh[lane] = h;
            eW[lane] = w;
            elo[lane] = lo;
            est[lane] = incl - cnt;
            efl[lane] = 0u;
            wave_lds_sync();
            for (int r = 0; r < total; r += 64) {
                const int idx = r + lane;
                if (idx < total) {
                    const int k = owner_of(est, idx);
                    const int j = elo[k] + (idx - est[k]);
                    if (rowb[j] == mk_prev && (sX[j] ^ eh[k]) < eW[k]) {
                        uint8_t* p = a.M + (size_t)ev[k] * (size_t)J + (size_t)j;
                        if (uncovered(*p)) {
                            *p = mk_cur;
                            efl[k] = 1u;
                        }
                    }
                }
            }
            wave_lds_sync();
            bool push_q = false, push_t = false;
            if (efl[lane]) {
                push_q = atomicMax(&a.c.stamp[v], a.level_id) < a.level_id;
                push_t = atomicMax(&a.c.touch_stamp[v], a.cascade_id) < a.cascade_id;
            }
            wave_append(push_q, v, Qn, qn_ctr);
            wave_append(push_t, v, a.c.touched, a.c.ntouched);
            wave_lds_sync();
        }
    }
}

hipError_t launch_cascade_level(const GraphDev& g, const uint32_t* X, int J, uint8_t* M, const CascadeDev& c, int t,
                                uint32_t level_id, uint32_t cascade_id, hipStream_t st)
{
    static int grid = 0;
    LevelArgs a{g, X, J, M, c, t, level_id, cascade_id};
    const size_t lds = sizeof(uint32_t) * ((size_t)J + (size_t)kWaves * ((size_t)(J / 4) + kLevelBufWords));
    if (grid == 0) {
        hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cascade_level),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
        if (err != hipSuccess) return err;
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = cus * 4;
    }
    hipLaunchKernelGGL(k_cascade_level, dim3(grid), dim3(kWG), lds, st, a);
    return hipGetLastError();
}

// End of a cascade: markers become 0 in every touched row; Ju/Hu of touched
// rows are recomputed and T grows by the number of newly covered registers.
__global__ __launch_bounds__(kWG) void k_cascade_finalize(uint8_t* M, int J, uint32_t* Ju, unsigned long long* Hu,
                                                           CascadeDev c)
{
    const int lane = lane_id();
    const int Jw = J >> 2;
    const uint32_t nt = *c.ntouched;
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t i = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); i < (int64_t)nt; i += nw) {
        const int32_t v = c.touched[i];
        uint32_t* row = reinterpret_cast<uint32_t*>(M + (size_t)v * (size_t)J);
        uint32_t cnt = 0;
        unsigned long long h = 0;
        for (int idx = lane; idx < Jw; idx += 64) {
            uint32_t d = row[idx], o = d;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                uint32_t r = (d >> (8 * b)) & 0xffu;
                if (r >= 64u) {
                    d &= ~(0xffu << (8 * b));
                } else if (r) {
                    ++cnt;
                    h += 1ull << (33u - r);
                }
            }
            if (d != o) row[idx] = d;
        }
        cnt = wave_sum_u32(cnt);
        h = wave_sum_u64(h);
        if (lane == 0) {
            uint32_t old = Ju[v];
            Ju[v] = cnt;
            Hu[v] = h;
            atomicAdd(c.T, (unsigned long long)(old - cnt));
        }
    }
}

hipError_t launch_cascade_finalize(uint8_t* M, int J, uint32_t* Ju, unsigned long long* Hu, const CascadeDev& c,
                                   hipStream_t st)
{
    static int grid = 0;
    if (grid == 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = cus * 4;
    }
    hipLaunchKernelGGL(k_cascade_finalize, dim3(grid), dim3(kWG), 0, st, M, J, Ju, Hu, c);
    return hipGetLastError();
}

}  // namespace imx
