// HIP kernels for gfx950 (MI355X): fused hash sampling, register fill,
// pull-based propagation, estimate, argmax and the union-frontier cascade.
//
// Register layout: M is uint8[n][J], vertex-major, registers of a row in
// increasing (sorted-X) simulation order.  Uncovered registers hold
// rank values 1..33; covered registers hold 0.  During a cascade, registers
// covered at frontier level t temporarily hold the marker 64 + (t mod 64).
#include "imx_internal.h"

#include <hip/hip_runtime.h>

#include <cstdlib>
#include <mutex>

namespace imx {

// ---------------------------------------------------------------------------
// MurmurHash3_x86_32 pieces (published algorithm by A. Appleby).

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

// A key block as the hash mixes it in (depends on the block only).
__device__ __forceinline__ uint32_t key_block(uint32_t k)
{
    k *= 0xcc9e2d51u;
    k = rotl32(k, 15);
    return k * 0x1b873593u;
}

__device__ __forceinline__ uint32_t mix_key(uint32_t h, uint32_t kk)
{
    h ^= kk;
    h = rotl32(h, 13);
    return h * 5u + 0xe6546b64u;
}

__device__ __forceinline__ uint32_t mix_block(uint32_t h, uint32_t k) { return mix_key(h, key_block(k)); }

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

// Eq. 3 with the HyperLogLog offset: leading zeros of the j-th hash, plus
// one; kj = key_block(j).
__device__ __forceinline__ uint32_t rank_from_key(uint32_t prefix, uint32_t kj)
{
    const uint32_t g = finish(mix_key(prefix, kj), 16u);
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
// simulation lies in one contiguous index range [lo, hi) of X.  T is the
// bucket table T[k] = first index with X >= k * 2^21 (k = 0..1024): range ends
// that are multiples of 2^21 are exact lookups, others step through one
// bucket (about J/1024 entries).
__device__ __forceinline__ void candidate_range(const uint32_t* X, const uint32_t* T, int J, uint32_t h, uint32_t W,
                                                int& lo, int& hi)
{
    if (W == 0u) {
        lo = hi = 0;
    } else if (W >= 0x80000000u) {
        lo = 0;
        hi = J;
    } else {
        const int b = (W == 1u) ? 0 : 32 - __builtin_clz(W - 1u);
        const uint32_t base = (h >> b) << b;
        const uint32_t top = base + (1u << b);
        if (b >= kBucketShift) {
            lo = (int)T[base >> kBucketShift];
            hi = (int)T[top >> kBucketShift];
        } else {
            lo = (int)T[base >> kBucketShift];
            const int end = (int)T[(base >> kBucketShift) + 1];
            while (lo < end && X[lo] < base) ++lo;
            hi = lo;
            while (hi < end && X[hi] < top) ++hi;
        }
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

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Byte-wise max of four packed registers (values < 256): even and odd bytes
// are compared as two packed 16-bit lanes each.
__device__ __forceinline__ uint32_t bytemax4(uint32_t a, uint32_t b)
{
    const u16x2 ae = __builtin_bit_cast(u16x2, a & 0x00ff00ffu), be = __builtin_bit_cast(u16x2, b & 0x00ff00ffu);
    const u16x2 ao = __builtin_bit_cast(u16x2, (a >> 8) & 0x00ff00ffu);
    const u16x2 bo = __builtin_bit_cast(u16x2, (b >> 8) & 0x00ff00ffu);
    const uint32_t e = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(ae, be));
    const uint32_t o = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(ao, bo));
    return e | (o << 8);
}

// 0xff in byte b iff simulation x4[b] has the arc (hash h, threshold W) live (Eq. 2).
__device__ __forceinline__ uint32_t live_mask4(uint4 x4, uint32_t h, uint32_t W)
{
    return ((x4.x ^ h) < W ? 0x000000ffu : 0u) | ((x4.y ^ h) < W ? 0x0000ff00u : 0u) |
           ((x4.z ^ h) < W ? 0x00ff0000u : 0u) | ((x4.w ^ h) < W ? 0xff000000u : 0u);
}

// 0xff in byte b iff byte b of d equals v.
__device__ __forceinline__ uint32_t eq_mask4(uint32_t d, uint32_t v)
{
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        if (((d >> (8 * b)) & 0xffu) == v) m |= 0xffu << (8 * b);
    return m;
}

// 0xff in byte b iff byte b of d is an uncovered register (rank 1..33).
__device__ __forceinline__ uint32_t uncovered_mask4(uint32_t d)
{
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t r = (d >> (8 * b)) & 0xffu;
        if (r >= 1u && r <= 33u) m |= 0xffu << (8 * b);
    }
    return m;
}

__device__ __forceinline__ uint32_t pack4(uint4 w) { return w.x | (w.y << 8) | (w.z << 16) | (w.w << 24); }

// Per-wave staging buffer in LDS for appends to a global list: ids appended by
// the lanes are collected and written out in batches, so the list's counter
// takes one atomic per batch instead of one per append.
constexpr int kWaveBufCap = 256;

// Value of x in lane l, l the same in every lane: a scalar read of the
// register instead of a permute through LDS.
__device__ __forceinline__ int lane_val(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ uint32_t lane_val(uint32_t x, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)x, l); }

struct WaveList {
    int32_t* buf;   // LDS staging area of `cap` entries
    int n;          // staged entries (wave-uniform)
    int32_t* L;     // global list
    uint32_t* ctr;  // global count
    int cap = kWaveBufCap;
};

__device__ __forceinline__ void wl_flush(WaveList& w)
{
    if (w.n == 0) return;
    wave_lds_sync();
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(w.ctr, (uint32_t)w.n);
    base = lane_val(base, 0);
    for (int i = lane_id(); i < w.n; i += 64) w.L[base + i] = w.buf[i];
    w.n = 0;
    wave_lds_sync();
}

// Append ids first..first+cnt-1 of every lane (cnt may differ per lane, 0 = none).
__device__ __forceinline__ void wl_append_ranges(WaveList& w, int cnt, int32_t first)
{
    const int lane = lane_id();
    const int incl = wave_incl_scan(cnt);
    const int total = lane_val(incl, 63);
    if (total == 0) return;
    if (total > w.cap) {
        uint32_t base = 0;
        if (lane == 63) base = atomicAdd(w.ctr, (uint32_t)total);
        base = lane_val(base, 63);
        const uint32_t off = base + (uint32_t)(incl - cnt);
        for (int q = 0; q < cnt; ++q) w.L[off + q] = first + q;
        return;
    }
    if (w.n + total > w.cap) wl_flush(w);
    const int off = w.n + incl - cnt;
    for (int q = 0; q < cnt; ++q) w.buf[off + q] = first + q;
    w.n += total;
}

// Append ids first..first+cnt-1 where cnt and first are the same in every lane.
__device__ __forceinline__ void wl_append_uniform(WaveList& w, int cnt, int32_t first)
{
    const int lane = lane_id();
    if (cnt <= 0) return;
    if (cnt > w.cap) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(w.ctr, (uint32_t)cnt);
        base = lane_val(base, 0);
        for (int q = lane; q < cnt; q += 64) w.L[base + q] = first + q;
        return;
    }
    if (w.n + cnt > w.cap) wl_flush(w);
    for (int q = lane; q < cnt; q += 64) w.buf[w.n + q] = first + q;
    w.n += cnt;
}

// End-of-kernel flush of the lists of every wave of the workgroup with one
// global atomic per workgroup (same-address atomics serialise at memory, so
// per-wave flushes of thousands of waves dominate short kernels).  Every
// thread of the workgroup must call it; all waves' lists share L and ctr.
// `tmp` is kWaves + 1 words of LDS.
__device__ __forceinline__ void wg_flush(WaveList& w, uint32_t* tmp)
{
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = lane_id();
    if (lane == 0) tmp[wave] = (uint32_t)w.n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int i = 0; i < kWaves; ++i) tot += tmp[i];
        tmp[kWaves] = tot ? atomicAdd(w.ctr, tot) : 0u;
    }
    __syncthreads();
    uint32_t base = tmp[kWaves];
    for (int i = 0; i < wave; ++i) base += tmp[i];
    for (int i = lane; i < w.n; i += 64) w.L[base + i] = w.buf[i];
    w.n = 0;
    __syncthreads();
}

// Sum of a per-wave 64-bit count over the workgroup, added to *ctr with one
// atomic (every thread must call; `tmp` is kWaves 64-bit words of LDS).
__device__ __forceinline__ void wg_add_u64(unsigned long long x, unsigned long long* ctr, unsigned long long* tmp)
{
    const int wave = (int)(threadIdx.x >> 6);
    x = wave_sum_u64(x);
    if (lane_id() == 0) tmp[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int i = 0; i < kWaves; ++i) tot += tmp[i];
        if (tot) atomicAdd(ctr, tot);
    }
    __syncthreads();
}

// Compaction of a per-vertex flag array (flag_bytes(n) bytes, 16 flags per
// lane): every flagged vertex v appends its out-tasks task_start[v] ..
// task_start[v+1]-1 to L and, with TOUCH, appends v itself to T unless
// touch_stamp[v] already holds `id` (then sets it).  The flags are cleared.
// Every vertex belongs to one lane, so flags and stamps need no atomics; the
// lists take one atomic per staged batch.  Wave-uniform control flow.
template <bool TOUCH>
__device__ __forceinline__ void compact_flags(uint8_t* flags, uint8_t* blk, int64_t n, const int32_t* task_start,
                                              WaveList& L, WaveList& T, uint32_t* touch_stamp, uint32_t id,
                                              int64_t first_wave, int64_t nwaves)
{
    static_assert(kFlagBlock == 64 * 16, "a wave's 64 chunks of 16 flags are one flag block");
    const int lane = lane_id();
    const int64_t nchunks = (n + 15) / 16;
    uint4* F = reinterpret_cast<uint4*>(flags);
    for (int64_t cb = first_wave * 64; cb < nchunks; cb += nwaves * 64) {
        // one block of flags per wave iteration; blocks without flags are skipped
        if (blk[cb >> 6] == 0u) continue;
        if (lane == 0) blk[cb >> 6] = 0u;
        const int64_t c = cb + lane;
        uint4 f = make_uint4(0u, 0u, 0u, 0u);
        if (c < nchunks) f = F[c];
        const bool any = (f.x | f.y | f.z | f.w) != 0u;
        if (__ballot(any) == 0ull) continue;
        // task ranges (and stamps) of the chunk's 16 vertices, loaded at once
        int32_t ts[17];
        uint32_t st[16];
#pragma unroll
        for (int b = 0; b < 17; ++b) ts[b] = 0;
#pragma unroll
        for (int b = 0; b < 16; ++b) st[b] = id;
        const int64_t v0 = c * 16;
        if (any) {
            F[c] = make_uint4(0u, 0u, 0u, 0u);
            if (v0 + 16 <= n) {
                const int4* p = reinterpret_cast<const int4*>(task_start + v0);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int4 q = p[k];
                    ts[4 * k] = q.x;
                    ts[4 * k + 1] = q.y;
                    ts[4 * k + 2] = q.z;
                    ts[4 * k + 3] = q.w;
                }
                ts[16] = task_start[v0 + 16];
                if (TOUCH) {
                    const uint4* ps = reinterpret_cast<const uint4*>(touch_stamp + v0);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint4 q = ps[k];
                        st[4 * k] = q.x;
                        st[4 * k + 1] = q.y;
                        st[4 * k + 2] = q.z;
                        st[4 * k + 3] = q.w;
                    }
                }
            } else {  // the last, partial chunk
#pragma unroll
                for (int b = 0; b < 17; ++b)
                    if (v0 + b <= n) ts[b] = task_start[v0 + b];
                if (TOUCH) {
#pragma unroll
                    for (int b = 0; b < 16; ++b)
                        if (v0 + b < n) st[b] = touch_stamp[v0 + b];
                }
            }
        }
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const uint32_t fw = (b < 4) ? f.x : (b < 8) ? f.y : (b < 12) ? f.z : f.w;
            const bool set = ((fw >> (8 * (b & 3))) & 0xffu) != 0u;
            if (__ballot(set) == 0ull) continue;
            const int32_t v = (int32_t)(v0 + b);
            const int cnt = set ? ts[b + 1] - ts[b] : 0;
            bool push = false;
            if (TOUCH && set && st[b] != id) {
                touch_stamp[v] = id;
                push = true;
            }
            wl_append_ranges(L, cnt, ts[b]);
            if (TOUCH) wl_append_ranges(T, push ? 1 : 0, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Batched launches: the workgroups of one launch are split among up to
// kMaxBatch queries (query i owns workgroups wg0[i] .. wg0[i+1]-1 and reads
// argument record args[i]); each workgroup works for exactly one query and
// strides over that query's work with its local index and local grid size.

__device__ __forceinline__ int batch_index(const Batch& B)
{
    int i = 0;
#pragma unroll
    for (int step = kMaxBatch / 2; step > 0; step >>= 1)
        if (i + step < B.nq && B.wg0[i + step] <= (int)blockIdx.x) i += step;
    return i;
}

// The kernels' view of a host-filled argument record (same layout; its
// pointers carry the global address space).
template <template <bool> class S>
__device__ __forceinline__ const S<true>& gview(const S<false>& x)
{
    return reinterpret_cast<const S<true>&>(x);
}

// Work of a record now (read from the device counters the earlier kernels of
// the step left), for the dynamic split below.
template <class R>
__device__ __forceinline__ unsigned long long work_weight(const R&) { return 1ull; }
__device__ __forceinline__ unsigned long long work_weight(const PropArgsT<true>& a)
{
    return (a.tasks == nullptr || *a.dense != 0u) ? (unsigned long long)a.g.ntasks : (unsigned long long)*a.task_count;
}
__device__ __forceinline__ unsigned long long work_weight(const LevelArgsT<true>& a)
{
    return a.c.qsize[a.t & 3];
}
__device__ __forceinline__ unsigned long long work_weight(const MarkArgsT<true>& a)
{
    return a.s.chg_count[a.sweep & 3];
}
__device__ __forceinline__ unsigned long long work_weight(const FillArgsT<true>& a) { return (unsigned long long)a.n; }
__device__ __forceinline__ unsigned long long work_weight(const EstArgsT<true>& a) { return (unsigned long long)a.n; }
__device__ __forceinline__ unsigned long long work_weight(const PrepArgsT<true>& a)
{
    return (unsigned long long)a.n >> 10;
}
__device__ __forceinline__ unsigned long long work_weight(const LevelCompactArgsT<true>& a)
{
    return (unsigned long long)a.n >> 10;
}
__device__ __forceinline__ unsigned long long work_weight(const FinArgsT<true>& a)
{
    return (*a.c.level_end != ~0u) ? (unsigned long long)*a.c.ntouched : 0ull;
}

// Dynamic split (B.wg0[0] == -1, B.wg0[B.nq] = the grid): the launch's
// workgroups are divided among the records at run time, each active record
// getting one plus a share of the rest in proportion to its current work, so
// a launch whose sequence is fixed (graph mode) spends no workgroups on
// queries without work in it.  Lane i of every wave computes record i's share
// (kMaxBatch = 64 records at most); every wave reaches the same split.  The
// host makes the grid at least the number of records.  Returns false for a
// workgroup left without a record.
template <class A>
__device__ __forceinline__ bool dyn_split(const A* args, const Batch& B, int& bi, int64_t& lb, int64_t& lg)
{
    static_assert(kMaxBatch <= 64, "one lane per record");
    const int lane = lane_id();
    unsigned long long w = 0ull;
    if (lane < B.nq) {
        const auto& r = gview(args[lane]);
        if (r.active) {
            const unsigned long long ww = work_weight(r);
            w = ww > 0ull ? ww : 1ull;
        }
    }
    const unsigned long long W = wave_sum_u64(w);
    const int nact = __popcll(__ballot(w > 0ull));
    const int64_t G = gridDim.x;
    const int64_t rest = G > nact ? G - nact : 0;
    const int blocks = (w > 0ull) ? 1 + (int)((unsigned long long)rest * w / (W > 0ull ? W : 1ull)) : 0;
    const int incl = wave_incl_scan(blocks);
    const int64_t start = incl - blocks;
    const int64_t b = blockIdx.x;
    const unsigned long long mine = __ballot(blocks > 0 && b >= start && b < (int64_t)incl);
    if (mine == 0ull) return false;
    const int l = __ffsll((long long)mine) - 1;
    bi = l;
    lb = b - lane_val((int)start, l);
    lg = lane_val(blocks, l);
    return true;
}

#define IMX_BATCH_PROLOGUE(ArgsT)                                     \
    int bi_ = 0;                                                      \
    int64_t lb = 0, lg = 1;                                           \
    if (B.wg0[0] < 0) {                                               \
        if (!dyn_split(args, B, bi_, lb, lg)) return;                 \
    } else {                                                          \
        bi_ = batch_index(B);                                         \
        lb = (int64_t)blockIdx.x - B.wg0[bi_];                        \
        lg = (int64_t)B.wg0[bi_ + 1] - B.wg0[bi_];                    \
    }                                                                 \
    const auto& a = gview(args[bi_]);                                 \
    (void)lb;                                                         \
    (void)lg;                                                         \
    if (!a.active) return

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
    for (int k = threadIdx.x; k <= kBuckets; k += blockDim.x)
        X[J + k] = (uint32_t)lower_bound_lds(s, J, (uint32_t)k << kBucketShift);
}

hipError_t launch_sim_values(uint64_t seed, int J, uint32_t* X, hipStream_t st)
{
    hipLaunchKernelGGL(k_sim_values, dim3(1), dim3(1024), 0, st, seed, J, X);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a3: Fill-Sketches (Alg. 1).  One thread per 4 registers.  On a rebuild,
// covered registers (0) stay 0.



// Registers of one 16-byte chunk (simulations 16c .. 16c+15) of a row with
// rank prefix `pre`; covered registers (0 in `old`) stay 0.
__device__ __forceinline__ uint4 fill_chunk(uint32_t pre, const uint32_t (&kj)[16], uint4 old)
{
    const uint32_t ow[4] = {old.x, old.y, old.z, old.w};
    uint32_t out[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t r = ((ow[w] >> (8 * b)) & 0xffu) ? rank_from_key(pre, kj[4 * w + b]) : 0u;
            o |= r << (8 * b);
        }
        out[w] = o;
    }
    return make_uint4(out[0], out[1], out[2], out[3]);
}

__global__ __launch_bounds__(256) void k_fill(const FillArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(FillArgs);
    const int L = row_lanes(a.J);
    const int sub = lane_id() % L;
    const int chunks = a.J / 16;  // per row
    const int64_t rows_per_iter = (int64_t)lg * (blockDim.x / L);
    uint4* M4 = reinterpret_cast<uint4*>(a.M);
    // key blocks of the lane's first chunk, reused for every row
    uint32_t kj0[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) kj0[b] = key_block((uint32_t)(16 * sub + b));
    const uint4 all_uncovered = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (int64_t u = lb * (blockDim.x / L) + threadIdx.x / L; u < a.n; u += rows_per_iter) {
        const uint32_t pre = rank_prefix(a.seed, (uint32_t)u);
        uint4* row = M4 + (size_t)u * (size_t)chunks;
        if (sub < chunks) row[sub] = fill_chunk(pre, kj0, a.first ? all_uncovered : row[sub]);
        for (int c = sub + L; c < chunks; c += L) {
            uint32_t kj[16];
#pragma unroll
            for (int b = 0; b < 16; ++b) kj[b] = key_block((uint32_t)(16 * c + b));
            row[c] = fill_chunk(pre, kj, a.first ? all_uncovered : row[c]);
        }
    }
}

hipError_t launch_fill(const FillArgs* args, const Batch& B, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3(B.wg0[B.nq]), dim3(256), 0, st, args, B);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a4: propagation sweeps (Alg. 2, pull-based, in place), frontier-driven.
//
// Work unit: a task = a vertex u, or a run of at most `split` of its out-arcs.
// Each wave is cut into lane groups of GS lanes (GS = 16, 32 or 64); every
// group owns one task, so a wave has 64/GS independent dependency chains in
// flight.  Per task:
//   - lane-per-arc phase: for arcs whose head v changed in the previous sweep,
//     the arc hash (Eq. 1), threshold, and the candidate range [lo, hi) of
//     sorted X that holds every simulation the arc can be live in;
//   - u's row is staged in LDS as bytes; dense arcs (at least J/2 candidates)
//     are merged by the whole group, each lane owning fixed 32-bit words;
//     sparse arcs are flattened into (arc, word) items dealt to the group's
//     lanes.  Every merge is a byte-wise max (Eq. 5) of the head's word masked
//     to the simulations where the arc is live (Eq. 2).  Items of one round may
//     hit the same LDS word; a read-max-write-verify loop settles them (the
//     last writer among colliding lanes exits each round, so it terminates);
//   - changed words (tracked in a per-group dirty bitmap) are stored to HBM;
//     rows split over several tasks merge with a byte-max compare-and-swap.
//     A changed row u is flagged in the next changed bitmap and its in-tasks
//     are queued; k_mark turns them into the next sweep's active task list,
//     unless so many rows changed that the next sweep visits every task.



constexpr int kPropBufCap = 256;  // staging entries per wave for the changed in-task list

// LDS words per group besides the row: arc arrays (5 x GS), dirty bitmap
// (Jw/32 <= 32 words), and (instrumented variant) sector masks (2 x GS).
template <int GS, bool STATS>
constexpr int group_buf_words()
{
    return 5 * GS + 32 + (STATS ? 2 * GS : 0);
}

__device__ __forceinline__ unsigned long long group_mask(int gbase, int GS)
{
    return (GS == 64) ? ~0ull : (((1ull << GS) - 1ull) << gbase);
}

template <int GS>
__device__ __forceinline__ int group_incl_scan(int x, int lig)
{
#pragma unroll
    for (int d = 1; d < GS; d <<= 1) {
        int y = __shfl_up(x, d, GS);
        if (lig >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ int wave_max_i32(int x)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const int y = __shfl_xor(x, d, 64);
        x = x > y ? x : y;
    }
    return x;
}

// Largest k in [0,GS) with start[k] <= idx (start non-decreasing, start[0] = 0).
template <int GS>
__device__ __forceinline__ int group_owner(const int* start, int idx)
{
    int k = 0;
#pragma unroll
    for (int step = GS / 2; step > 0; step >>= 1)
        if (start[k + step] <= idx) k += step;
    return k;
}

// Byte-wise max of `val` into LDS word w (index d) for lanes with `pending`;
// lanes of one wave may collide on a word.  Each pass, every colliding lane
// whose value the word already dominates leaves, and the lane whose write
// landed last always does, so the loop ends after at most 64 passes.
__device__ __forceinline__ void lds_merge_word(uint32_t* w, uint32_t* dirty, int d, uint32_t val, bool pending)
{
    while (__ballot(pending) != 0ull) {
        if (pending) {
            const uint32_t cur = *w;
            const uint32_t want = bytemax4(cur, val);
            if (want == cur) {
                pending = false;
            } else {
                *w = want;
                atomicOr(&dirty[d >> 5], 1u << (d & 31));
            }
        }
        wave_lds_sync();
    }
}

// Items (arc, word) each lane of a group gathers per round of the sparse merge.
constexpr int kItemsPerLane = 2;

// Six waves per SIMD: the kernel is bound by the latency of dependent
// gathers, and this is the most waves that fit without register spills.
// As lds_merge_word, with the changed word recorded as a dirty byte (plain
// LDS byte stores: no atomics on shared dirty words).
__device__ __forceinline__ void lds_merge_word8(uint32_t* w, uint8_t* dirty8, int d, uint32_t val, bool pending)
{
    while (__ballot(pending) != 0ull) {
        if (pending) {
            const uint32_t cur = *w;
            const uint32_t want = bytemax4(cur, val);
            if (want == cur) {
                pending = false;
            } else {
                *w = want;
                dirty8[d] = 1u;
            }
        }
        wave_lds_sync();
    }
}

template <int GS, int DPLG, bool STATS>
__global__ __launch_bounds__(kWG, 6) void k_propagate(const PropArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(PropArgs);
    constexpr int NG = 64 / GS;
    constexpr int GB = group_buf_words<GS, STATS>();
    extern __shared__ uint32_t smem[];
    const int J = a.J;
    const int Jw = J >> 2;
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = lane_id();
    const int gi = lane / GS, lig = lane % GS, gbase = gi * GS;
    const unsigned long long gmask = group_mask(gbase, GS);

    uint32_t* sX = smem;
    const uint32_t* sT = smem + J;
    const int XT = J + kTableWords;
    int32_t* wbuf = reinterpret_cast<int32_t*>(smem + XT + wave * kPropBufCap);
    uint32_t* gbuf = smem + XT + kWaves * kPropBufCap + (wave * NG + gi) * (Jw + GB);
    uint32_t* rowW = gbuf;  // Jw words = J register bytes
    int* ev = reinterpret_cast<int*>(gbuf + Jw);
    uint32_t* eh = gbuf + Jw + GS;
    uint32_t* eW = gbuf + Jw + 2 * GS;
    int* edl = reinterpret_cast<int*>(gbuf + Jw + 3 * GS);
    int* est = reinterpret_cast<int*>(gbuf + Jw + 4 * GS);
    uint32_t* dirty = gbuf + Jw + 5 * GS;
    unsigned long long* esec = reinterpret_cast<unsigned long long*>(gbuf + Jw + 5 * GS + 32);  // STATS only
    WaveList chl{wbuf, 0, a.chg_list, a.chg_count, kPropBufCap};
    unsigned long long c_tasks = 0, c_rows = 0, c_wbytes = 0, c_scanned = 0, c_active = 0, c_sectors = 0;
    unsigned long long c_changed = 0, c_visited = 0;

    const auto& g = a.g;
    // every task after a fill or after a sweep that changed many rows; else the active list
    const bool sweep0 = a.tasks == nullptr;  // right after a fill every head counts as changed
    const bool all = sweep0 || *a.dense != 0u;
    const int32_t* tasks = all ? nullptr : a.tasks;
    const int64_t count = all ? g.ntasks : (int64_t)*a.task_count;
    const int64_t ngroups = lg * kWaves * NG;
    if (*a.conv != ~0u) return;             // the build has converged
    if (lb * kWaves * NG >= count) return;  // no task for this workgroup (uniform)

    for (int i = threadIdx.x; i < J + kBuckets + 1; i += kWG) sX[i] = a.X[i];
    __syncthreads();

    const uint32_t* M32 = reinterpret_cast<const uint32_t*>(a.M);
    uint32_t* MW = reinterpret_cast<uint32_t*>(a.M);
    const uint32_t* chg_prev = a.chg_prev;

    // The id of the group's next task is loaded one iteration ahead.
    int64_t qb = (lb * kWaves + wave) * NG;
    int32_t t_next = -1;
    if (qb + gi < count) t_next = tasks ? tasks[qb + gi] : (int32_t)(qb + gi);

    for (; qb < count; qb += ngroups) {
        const int32_t t = t_next;
        const bool valid = t >= 0;
        int32_t u = 0;
        int64_t e0 = 0, e1 = 0;
        bool split = false;
        if (valid) {
            u = g.task_u[t];
            e0 = g.task_e0[t];
            const uint32_t len = g.task_len[t];
            e1 = e0 + (int64_t)(len & 0x7fffffffu);
            split = (len >> 31) != 0u;
        }
        {
            const int64_t qn = qb + ngroups + gi;
            t_next = -1;
            if (qn < count) t_next = tasks ? tasks[qn] : (int32_t)qn;
        }
        if (STATS && valid && lig == 0) ++c_tasks;
        const int nch = valid ? (int)((e1 - e0 + GS - 1) / GS) : 0;
        const int maxch = wave_max_i32(nch);

        // Independent loads issued together: u's row, the first chunk of
        // arcs, and u's in-task range (used only if the row changes).
        uint32_t rw[DPLG];
        const uint32_t* Mu = M32 + (size_t)u * (size_t)Jw;
#pragma unroll
        for (int i = 0; i < DPLG; ++i) {
            const int idx = lig + GS * i;
            rw[i] = (valid && idx < Jw) ? Mu[idx] : 0u;
        }
        int32_t v_nx = 0;
        uint32_t w_nx = 0;
        if (e0 + lig < e1) {
            v_nx = g.col[e0 + lig];
            w_nx = g.W[e0 + lig];
        }
        int32_t in_first = 0, in_cnt = 0;
        if (valid && lig == 0) {
            in_first = g.in_task_start[u];
            in_cnt = g.in_task_start[u + 1] - in_first;
        }
        if (valid) {
#pragma unroll
            for (int i = 0; i < DPLG; ++i) {
                const int idx = lig + GS * i;
                if (idx < Jw) rowW[idx] = rw[i];
            }
            if (lig < 32) dirty[lig] = 0u;
            if (GS == 16) dirty[lig + 16] = 0u;
        }
        bool touched = false;      // group-uniform: some arc had candidates
        bool task_active = false;  // group-uniform: some arc's head changed (instrumented variant)
        for (int c = 0; c < maxch; ++c) {
            const int64_t e = e0 + (int64_t)c * GS + lig;
            int cnt = 0, lo = 0, hi = 0;
            const int32_t v = v_nx;
            const uint32_t w = w_nx;
            uint32_t h = 0;
            if (c + 1 < maxch) {  // next chunk's arcs
                const int64_t en = e + GS;
                v_nx = 0;
                w_nx = 0;
                if (en < e1) {
                    v_nx = g.col[en];
                    w_nx = g.W[en];
                }
            }
            bool act_arc = false;
            if (e < e1) {
                act_arc = sweep0 || ((chg_prev[(uint32_t)v >> 5] >> (v & 31)) & 1u);
                if (act_arc && w != 0u) {
                    h = arc_hash((uint32_t)u, (uint32_t)v);
                    candidate_range(sX, sT, J, h, w, lo, hi);
                    cnt = hi - lo;
                }
            }
            if (STATS) {
                c_scanned += (e < e1) ? 1ull : 0ull;
                c_active += act_arc ? 1ull : 0ull;
                task_active |= (__ballot(act_arc) & gmask) != 0ull;
            }
            const bool gany = (__ballot(cnt > 0) & gmask) != 0ull;
            if (gany && !touched) {
                touched = true;
                if (STATS && lig == 0) ++c_rows;
            }
            const bool dense = cnt > 0 && 2 * cnt >= J;
            const int nd = (cnt > 0 && !dense) ? (((hi - 1) >> 2) - (lo >> 2) + 1) : 0;
            wave_lds_sync();

            // dense arcs: the group merges v's row word by word (each lane owns
            // fixed words, so no collisions); DB arcs' loads are in flight at once
            // (one measured best: more raise register pressure past the occupancy target)
            constexpr int DB = 1;
            unsigned long long rem = (__ballot(dense) & gmask) >> gbase;
            const int maxd = wave_max_i32(__popcll(rem));
            for (int k = 0; k < maxd; k += DB) {
                bool has[DB];
                int vk[DB], lok[DB], hik[DB];
                uint32_t hk[DB], wk[DB];
                uint32_t sv[DB][DPLG];
#pragma unroll
                for (int x = 0; x < DB; ++x) {
                    has[x] = rem != 0ull;
                    const int ak = has[x] ? __ffsll((long long)rem) - 1 : 0;
                    rem &= rem - 1ull;
                    vk[x] = __shfl(v, gbase + ak, 64);
                    hk[x] = __shfl(h, gbase + ak, 64);
                    wk[x] = __shfl(w, gbase + ak, 64);
                    lok[x] = __shfl(lo, gbase + ak, 64);
                    hik[x] = __shfl(hi, gbase + ak, 64);
                    const uint32_t* src = M32 + (size_t)vk[x] * (size_t)Jw;
#pragma unroll
                    for (int i = 0; i < DPLG; ++i) {
                        const int idx = lig + GS * i;
                        sv[x][i] = (has[x] && idx < Jw && 4 * idx + 3 >= lok[x] && 4 * idx < hik[x]) ? src[idx] : 0u;
                    }
                }
#pragma unroll
                for (int x = 0; x < DB; ++x) {
                    if (!has[x]) continue;
#pragma unroll
                    for (int i = 0; i < DPLG; ++i) {
                        const int idx = lig + GS * i;
                        if (idx < Jw && 4 * idx + 3 >= lok[x] && 4 * idx < hik[x]) {
                            const uint32_t val =
                                sv[x][i] & live_mask4(*reinterpret_cast<const uint4*>(&sX[4 * idx]), hk[x], wk[x]);
                            const uint32_t cur = rowW[idx];
                            const uint32_t want = bytemax4(cur, val);
                            if (want != cur) {
                                rowW[idx] = want;
                                atomicOr(&dirty[idx >> 5], 1u << (idx & 31));
                            }
                        }
                    }
                    if (STATS && lig == 0)
                        c_sectors += (unsigned long long)(((hik[x] - 1) >> 6) - (lok[x] >> 6) + 1);
                }
            }

            // sparse arcs: flattened (arc, word) items within the group
            const int incl = group_incl_scan<GS>(nd, lig);
            const int total = __shfl(incl, gbase + GS - 1, 64);
            const int maxtot = wave_max_i32(total);
            if (maxtot == 0) continue;
            ev[lig] = v;
            eh[lig] = h;
            eW[lig] = w;
            edl[lig] = lo >> 2;
            est[lig] = incl - nd;
            if (STATS) esec[lig] = 0ull;
            wave_lds_sync();
            for (int r = 0; r < maxtot; r += kItemsPerLane * GS) {
                uint32_t val[kItemsPerLane];
                int dw[kItemsPerLane];
#pragma unroll
                for (int x = 0; x < kItemsPerLane; ++x) {
                    const int ii = r + x * GS + lig;
                    val[x] = 0u;
                    dw[x] = 0;
                    if (ii < total) {
                        const int k = group_owner<GS>(est, ii);
                        dw[x] = edl[k] + (ii - est[k]);
                        const uint32_t m = live_mask4(*reinterpret_cast<const uint4*>(&sX[4 * dw[x]]), eh[k], eW[k]);
                        if (m) {
                            val[x] = M32[(size_t)ev[k] * (size_t)Jw + (size_t)dw[x]] & m;
                            if (STATS) atomicOr(&esec[k], 1ull << ((4 * dw[x]) >> 6));
                        }
                    }
                }
#pragma unroll
                for (int x = 0; x < kItemsPerLane; ++x) lds_merge_word(&rowW[dw[x]], dirty, dw[x], val[x], val[x] != 0u);
            }
            if (STATS) {
                c_sectors += (unsigned long long)__popcll(esec[lig]);
            }
            wave_lds_sync();
        }

        wave_lds_sync();
        // store changed words of u's row
        bool changed = false;
        if (touched) {
            uint32_t* Mw = MW + (size_t)u * (size_t)Jw;
#pragma unroll
            for (int i = 0; i < DPLG; ++i) {
                const int idx = lig + GS * i;
                if (idx < Jw && ((dirty[idx >> 5] >> (idx & 31)) & 1u)) {
                    const uint32_t nwd = rowW[idx];
                    if (!split) {
                        Mw[idx] = nwd;
                        changed = true;
                        if (STATS) c_wbytes += 4;
                    } else {
                        uint32_t cur = Mw[idx];
                        for (;;) {
                            const uint32_t want = bytemax4(cur, nwd);
                            if (want == cur) break;
                            const uint32_t prev = atomicCAS(&Mw[idx], cur, want);
                            if (prev == cur) {
                                changed = true;
                                if (STATS) c_wbytes += 4;
                                break;
                            }
                            cur = prev;
                        }
                    }
                }
            }
        }
        const bool gchanged = (__ballot(changed) & gmask) != 0ull;
        // Flag u once per sweep; the first flagger queues u's in-tasks.  A
        // row with one task has one flagger, so its flag needs no reply.
        bool first = false;
        if (gchanged && lig == 0) {
            const uint32_t bit = 1u << (u & 31);
            if (!split) {
                atomicOr(&a.chg_next[(uint32_t)u >> 5], bit);
                first = true;
            } else {
                first = !(atomicOr(&a.chg_next[(uint32_t)u >> 5], bit) & bit);
            }
        }
        if (first) ++c_changed;
        if (STATS && task_active && lig == 0 && atomicMax(&a.vstamp[u], a.stamp_id) < a.stamp_id) ++c_visited;
        wl_append_ranges(chl, first ? in_cnt : 0, in_first);
    }
    // per-wave flushes here: measured faster than a workgroup-wide flush,
    // whose barrier holds finished waves until the slowest one of the group
    wl_flush(chl);
    {
        const unsigned long long tot = wave_sum_u64(c_changed);
        if (lane == 0 && tot) atomicAdd(a.rows_changed, tot);
    }
    if (STATS) {
        c_wbytes = wave_sum_u64(c_wbytes);
        c_tasks = wave_sum_u64(c_tasks);
        c_rows = wave_sum_u64(c_rows);
        c_scanned = wave_sum_u64(c_scanned);
        c_active = wave_sum_u64(c_active);
        c_sectors = wave_sum_u64(c_sectors);
        c_visited = wave_sum_u64(c_visited);
        const unsigned long long chg_tot = wave_sum_u64(c_changed);
        if (lane == 0) {
            atomicAdd(&a.stats->rows_visited, c_visited);
            atomicAdd(&a.stats->rows_changed, chg_tot);
            atomicAdd(&a.stats->tasks, c_tasks);
            atomicAdd(&a.stats->rows_read, c_rows);
            atomicAdd(&a.stats->bytes_written, c_wbytes);
            atomicAdd(&a.stats->arcs_scanned, c_scanned);
            atomicAdd(&a.stats->arcs_active, c_active);
            atomicAdd(&a.stats->sectors, c_sectors);
        }
    }
}

// ---------------------------------------------------------------------------
// Packed variant of the propagation: each wave takes a pack of P consecutive
// entries of the task list (P = 2048 / J rows, at least 1, at most 16) and
// stages all P rows of u in LDS; the pack's arcs are flattened over the 64
// lanes, so the fixed costs of a task (record and row loads, scans, the store
// and the flagging) are paid once per pack and lanes stay busy on small
// tasks.  Every merge is the same byte-wise max as in k_propagate; results
// are identical (the fixed point does not depend on the schedule).


// The workgroup's LDS layout (X table, then per wave: rows, dirty bytes, arc
// and task records, sector masks, list buffer) is defined in pack_layout.h;
// every configuration the launch code can form keeps the alignments the
// kernel's vector and 64-bit atomic LDS accesses need.
static_assert(pack_layouts_ok(), "packed-propagation LDS layout misaligned or too large");

int pack_bytes()
{
    static const int pb = [] {
        const char* v = std::getenv("IMX_PACK_BYTES");
        const int b = v ? std::atoi(v) : 2048;
        return (b == 1024 || b == 2048 || b == 4096) ? b : 2048;
    }();
    return pb;
}

// Eight waves per workgroup share the X table and the pack counter.  Six
// waves per SIMD: the LDS of a workgroup (about 46 KB at J = 512 with 2 KB
// packs) admits three workgroups per CU, and registers are held to that
// occupancy's share (measured faster than five waves with more registers, and
// than seven or eight waves with spills).
// The body works for workgroup lb of lg workgroups assigned to one query;
// the single-workgroup tail sweeps call it too.  LDS: pack_lds_words(maxJ,
// pb, STATS) words from the start of the dynamic area.
template <bool STATS>
__device__ __forceinline__ void propagate_pack_body(const PropArgsT<true>& a, int64_t lb, int64_t lg, int maxJ, int pb)
{
    extern __shared__ uint32_t smem[];
    const int J = a.J;
    const int Jw = J >> 2;
    const int P = pack_rows(J, pb);
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = lane_id();

    const auto& g = a.g;
    const bool sweep0 = a.tasks == nullptr;
    const bool all = sweep0 || *a.dense != 0u;
    const int32_t* tasks = all ? nullptr : a.tasks;
    const int64_t count = all ? g.ntasks : (int64_t)*a.task_count;
    const int64_t npacks = (count + P - 1) / P;
    if (*a.conv != ~0u) return;                // the build has converged
    if (lb >= npacks) return;                   // no pack for this workgroup (uniform)

    uint32_t* sX = smem;
    const uint32_t* sT = smem + J;
    const int rw = pack_row_words(maxJ, pb), dw8 = pack_dirty_words(maxJ, pb);
    uint32_t* wbase = smem + pack_wave_base(maxJ, pb, STATS, wave);
    uint32_t* rows = wbase;                                      // P x Jw words
    uint8_t* dirty8 = reinterpret_cast<uint8_t*>(rows + rw);     // P x Jw bytes
    int* ev = reinterpret_cast<int*>(rows + rw + dw8);
    uint32_t* eh = reinterpret_cast<uint32_t*>(ev + 64);
    uint32_t* eW = eh + 64;
    int* edl = reinterpret_cast<int*>(eW + 64);
    int* est = edl + 64;
    int* ek = est + 64;
    int* T_u = ek + 64;
    uint32_t* T_e0lo = reinterpret_cast<uint32_t*>(T_u + kPackMax);
    uint32_t* T_e0hi = T_e0lo + kPackMax;
    int* T_pre = reinterpret_cast<int*>(T_e0hi + kPackMax);  // kPackMax + 1
    int* T_split = T_pre + kPackMax + 1;
    int* T_touch = T_split + kPackMax;
    int* T_act = T_touch + kPackMax;
    int* T_chg = T_act + kPackMax;
    int* T_in0 = T_chg + kPackMax;
    int* T_inc = T_in0 + kPackMax;
    unsigned long long* esec =
        reinterpret_cast<unsigned long long*>(smem + pack_esec_word(maxJ, pb, STATS, wave));  // STATS only; 8-byte aligned
    int32_t* wbuf = reinterpret_cast<int32_t*>(STATS ? reinterpret_cast<uint32_t*>(esec + 64)
                                                     : reinterpret_cast<uint32_t*>(esec));
    WaveList chl{wbuf, 0, a.chg_list, a.chg_count, kPackBufCap};
    unsigned long long c_tasks = 0, c_rows = 0, c_wbytes = 0, c_scanned = 0, c_active = 0, c_sectors = 0;
    unsigned long long c_changed = 0, c_visited = 0;

    // next draw of this workgroup's pack sequence: a padding word after the table
    uint32_t* const s_next = smem + (J + kBuckets + 1);
    if (threadIdx.x == 0) *s_next = 2 * kPackWaves;
    for (int i = threadIdx.x; i < J + kBuckets + 1; i += kPackWG) sX[i] = a.X[i];
    __syncthreads();

    const uint32_t* M32 = reinterpret_cast<const uint32_t*>(a.M);
    uint32_t* MW = reinterpret_cast<uint32_t*>(a.M);
    const uint4* M4 = reinterpret_cast<const uint4*>(a.M);
    const uint32_t* chg_prev = a.chg_prev;
    const int chunks16 = J / 16;  // 16-byte chunks per row
    const int dchunks = (P * Jw + 15) / 16;  // 16-byte chunks of the dirty bytes

    // Task records are loaded one pack ahead and task ids two packs ahead
    // (lanes 0..P-1 hold the pack's tasks).
    auto task_id = [&](int64_t pk) -> int32_t {
        const int64_t q = pk * P + lane;
        return (lane < P && pk < npacks && q < count) ? (tasks ? tasks[q] : (int32_t)q) : -1;
    };
    // task records: by task id from a list, or by position in the dense order
    const auto rec_u = tasks ? g.task_u : g.dense_u;
    const auto rec_e0 = tasks ? g.task_e0 : g.dense_e0;
    const auto rec_len = tasks ? g.task_len : g.dense_len;
    // Draw k of a workgroup is pack lb + k * lg (workgroups interleaved over
    // the list).  A wave's first two draws are fixed (k = wave, wave + 8);
    // later ones come from the workgroup's LDS counter, so the waves of a
    // workgroup share its packs dynamically and a wave that met cheap packs
    // takes more.  (A device-wide counter was measured 3-5x slower: atomics
    // on one global address serialise.)  A draw is made two packs ahead and
    // its task ids are loaded one pack ahead.
    auto pack_of = [&](uint32_t k) -> int64_t { return lb + (int64_t)k * lg; };
    auto draw = [&]() -> uint32_t {
        uint32_t r = 0u;
        if (lane == 0) r = atomicAdd(s_next, 1u);
        return r;
    };
    int64_t pk = pack_of((uint32_t)wave);
    int64_t pk_n1 = pack_of((uint32_t)(wave + kPackWaves)), pk_n2 = npacks;
    uint32_t drawn = (pack_of(2 * kPackWaves) < npacks) ? draw() : ~0u;  // lane 0: the draw after pk_n1
    int32_t t_nx = task_id(pk);
    int32_t u_nx = 0;
    int64_t e0_nx = 0;
    uint32_t len_nx = 0;
    if (t_nx >= 0) {
        u_nx = rec_u[t_nx];
        e0_nx = rec_e0[t_nx];
        len_nx = rec_len[t_nx];
    }
    int32_t t_nx2 = task_id(pk_n1);
    for (; pk < npacks; pk = pk_n1, pk_n1 = pk_n2) {
        const int32_t t = t_nx, u = u_nx;
        const int64_t e0 = e0_nx;
        const uint32_t len = len_nx;
        int in0 = 0, inc = 0;
        if (t >= 0) {
            in0 = g.in_task_start[u];
            inc = g.in_task_start[u + 1] - in0;
        }
        // next pack's records, and the ids of the one after
        t_nx = t_nx2;
        if (t_nx >= 0) {
            u_nx = rec_u[t_nx];
            e0_nx = rec_e0[t_nx];
            len_nx = rec_len[t_nx];
        }
        pk_n2 = pack_of(lane_val(drawn, 0));
        drawn = (pk_n2 < npacks) ? draw() : ~0u;  // wave-uniform
        t_nx2 = task_id(pk_n2);
        const int na = (t >= 0) ? (int)(len & 0x7fffffffu) : 0;
        const int incl = wave_incl_scan(na);
        const int A = lane_val(incl, 63);
        if (lane < P) {
            T_u[lane] = (t >= 0) ? u : -1;
            T_e0lo[lane] = (uint32_t)e0;
            T_e0hi[lane] = (uint32_t)((uint64_t)e0 >> 32);
            T_pre[lane] = incl - na;
            T_split[lane] = (len >> 31) ? 1 : 0;
            T_touch[lane] = 0;
            T_act[lane] = 0;
            T_chg[lane] = 0;
            T_in0[lane] = in0;
            T_inc[lane] = inc;
        }
        if (lane == 0) T_pre[P] = A;
        if (STATS && t >= 0) ++c_tasks;
        wave_lds_sync();
        // head id and threshold of arc ai of the pack (task k); the loads of
        // the next chunk are issued while the current one is processed, and
        // the first chunk's before the rows are staged
        auto arc_load = [&](int ai, int& k, int32_t& v, uint32_t& w) {
            k = 0;
            v = 0;
            w = 0;
            if (ai < A) {
#pragma unroll
                for (int step = kPackMax / 2; step > 0; step >>= 1)
                    if (k + step < P && T_pre[k + step] <= ai) k += step;
                const int64_t e = (int64_t)(((uint64_t)T_e0hi[k] << 32) | T_e0lo[k]) + (ai - T_pre[k]);
                v = g.col[e];
                w = g.W[e];
            }
        };
        int k_nx;
        int32_t v_nx;
        uint32_t w_nx;
        arc_load(lane, k_nx, v_nx, w_nx);
        // stage the P rows (16-byte chunks) and clear the dirty bits
        for (int c = lane; c < P * chunks16; c += 64) {
            const int k = c / chunks16, w = c - k * chunks16;
            const int uk = T_u[k];
            const uint4 d = (uk >= 0) ? M4[(size_t)uk * (size_t)chunks16 + w] : make_uint4(0u, 0u, 0u, 0u);
            reinterpret_cast<uint4*>(rows)[c] = d;
        }
        // changed-head words of the first chunk (its arcs came with the rows)
        uint32_t cw_nx = (lane < A && !sweep0) ? chg_prev[(uint32_t)v_nx >> 5] : ~0u;
        for (int i = lane; i < dchunks; i += 64) reinterpret_cast<uint4*>(dirty8)[i] = make_uint4(0u, 0u, 0u, 0u);
        wave_lds_sync();

        for (int base = 0; base < A; base += 64) {
            const int ai = base + lane;
            const int k = k_nx;
            const int32_t v = v_nx;
            const uint32_t w = w_nx;
            const uint32_t cw = cw_nx;
            // the next chunk's arcs are loaded while this one is processed (and
            // their changed-head words once the dense merges are issued); the
            // hash and candidate range are computed while loads are in flight
            if (base + 64 < A) arc_load(ai + 64, k_nx, v_nx, w_nx);
            int cnt = 0, lo = 0, hi = 0;
            uint32_t h = 0;
            // only arcs whose head changed in the previous sweep are hashed
            const bool act_arc = ai < A && ((cw >> (v & 31)) & 1u);
            if (act_arc && w != 0u) {
                h = arc_hash((uint32_t)T_u[k], (uint32_t)v);
                candidate_range(sX, sT, J, h, w, lo, hi);
            }
            cnt = hi - lo;
            if (ai < A) {
                if (STATS && act_arc) T_act[k] = 1;
                if (cnt > 0) T_touch[k] = 1;
            }
            if (STATS) {
                c_scanned += (ai < A) ? 1ull : 0ull;
                c_active += act_arc ? 1ull : 0ull;
            }
            const bool dense = cnt > 0 && 2 * cnt >= J;
            const int nd = (cnt > 0 && !dense) ? (((hi - 1) >> 2) - (lo >> 2) + 1) : 0;

            // dense arcs: the wave merges v's row word by word into row k
            unsigned long long rem = __ballot(dense);
            while (rem) {
                const int ak = __ffsll((long long)rem) - 1;
                rem &= rem - 1ull;
                const int vk = lane_val(v, ak), kk = lane_val(k, ak);
                const uint32_t hk = lane_val(h, ak), wk = lane_val(w, ak);
                const int lok = lane_val(lo, ak), hik = lane_val(hi, ak);
                const uint32_t* src = M32 + (size_t)vk * (size_t)Jw;
                uint32_t* rk = rows + kk * Jw;
                for (int idx = lane; idx < Jw; idx += 64) {
                    if (4 * idx + 3 >= lok && 4 * idx < hik) {
                        const uint32_t val = src[idx] & live_mask4(*reinterpret_cast<const uint4*>(&sX[4 * idx]), hk, wk);
                        const uint32_t cur = rk[idx];
                        const uint32_t want = bytemax4(cur, val);
                        if (want != cur) {
                            rk[idx] = want;
                            dirty8[kk * Jw + idx] = 1u;
                        }
                    }
                }
                if (STATS && lane == 0) c_sectors += (unsigned long long)(((hik - 1) >> 6) - (lok >> 6) + 1);
            }

            if (base + 64 < A) cw_nx = (ai + 64 < A && !sweep0) ? chg_prev[(uint32_t)v_nx >> 5] : ~0u;

            // sparse arcs: flattened (arc, word) items over the wave
            const int iincl = wave_incl_scan(nd);
            const int total = lane_val(iincl, 63);
            if (total == 0) continue;
            ev[lane] = v;
            eh[lane] = h;
            eW[lane] = w;
            edl[lane] = lo >> 2;
            est[lane] = iincl - nd;
            ek[lane] = k * Jw;
            if (STATS) esec[lane] = 0ull;
            wave_lds_sync();
            for (int r = 0; r < total; r += 2 * 64) {
                uint32_t val0 = 0u, val1 = 0u;
                int d0 = 0, d1 = 0;
                const int i0 = r + lane, i1 = r + 64 + lane;
                if (i0 < total) {
                    const int o = owner_of(est, i0);
                    const int dw = edl[o] + (i0 - est[o]);
                    d0 = ek[o] + dw;
                    const uint32_t m = live_mask4(*reinterpret_cast<const uint4*>(&sX[4 * dw]), eh[o], eW[o]);
                    if (m) {
                        val0 = M32[(size_t)ev[o] * (size_t)Jw + (size_t)dw] & m;
                        if (STATS) atomicOr(&esec[o], 1ull << ((4 * dw) >> 6));
                    }
                }
                if (i1 < total) {
                    const int o = owner_of(est, i1);
                    const int dw = edl[o] + (i1 - est[o]);
                    d1 = ek[o] + dw;
                    const uint32_t m = live_mask4(*reinterpret_cast<const uint4*>(&sX[4 * dw]), eh[o], eW[o]);
                    if (m) {
                        val1 = M32[(size_t)ev[o] * (size_t)Jw + (size_t)dw] & m;
                        if (STATS) atomicOr(&esec[o], 1ull << ((4 * dw) >> 6));
                    }
                }
                lds_merge_word8(&rows[d0], dirty8, d0, val0, val0 != 0u);
                lds_merge_word8(&rows[d1], dirty8, d1, val1, val1 != 0u);
            }
            if (STATS) c_sectors += (unsigned long long)__popcll(esec[lane]);
            wave_lds_sync();
        }
        wave_lds_sync();

        // store changed words of every row of the pack
        for (int idx = lane; idx < P * Jw; idx += 64) {
            if (!dirty8[idx]) continue;
            const int k = idx / Jw, d = idx - k * Jw;
            const uint32_t nwd = rows[idx];
            uint32_t* dst = MW + (size_t)T_u[k] * (size_t)Jw + d;
            if (!T_split[k]) {
                *dst = nwd;
                T_chg[k] = 1;
                if (STATS) c_wbytes += 4;
            } else {
                uint32_t cur = *dst;
                for (;;) {
                    const uint32_t want = bytemax4(cur, nwd);
                    if (want == cur) break;
                    const uint32_t prev = atomicCAS(dst, cur, want);
                    if (prev == cur) {
                        T_chg[k] = 1;
                        if (STATS) c_wbytes += 4;
                        break;
                    }
                    cur = prev;
                }
            }
        }
        wave_lds_sync();
        // flag changed rows once per sweep; the first flagger queues u's in-tasks
        bool first = false;
        if (lane < P && T_u[lane] >= 0 && T_chg[lane]) {
            const int uu = T_u[lane];
            const uint32_t bit = 1u << (uu & 31);
            if (!T_split[lane]) {
                atomicOr(&a.chg_next[(uint32_t)uu >> 5], bit);
                first = true;
            } else {
                first = !(atomicOr(&a.chg_next[(uint32_t)uu >> 5], bit) & bit);
            }
        }
        if (first) ++c_changed;
        if (STATS && lane < P && T_u[lane] >= 0) {
            if (T_touch[lane]) ++c_rows;
            if (T_act[lane] && atomicMax(&a.vstamp[T_u[lane]], a.stamp_id) < a.stamp_id) ++c_visited;
        }
        wl_append_ranges(chl, first ? T_inc[lane] : 0, lane < P ? T_in0[lane] : 0);
        wave_lds_sync();
    }
    wl_flush(chl);
    {
        const unsigned long long tot = wave_sum_u64(c_changed);
        if (lane == 0 && tot) atomicAdd(a.rows_changed, tot);
    }
    if (STATS) {
        c_wbytes = wave_sum_u64(c_wbytes);
        c_tasks = wave_sum_u64(c_tasks);
        c_rows = wave_sum_u64(c_rows);
        c_scanned = wave_sum_u64(c_scanned);
        c_active = wave_sum_u64(c_active);
        c_sectors = wave_sum_u64(c_sectors);
        c_visited = wave_sum_u64(c_visited);
        const unsigned long long chg_tot = wave_sum_u64(c_changed);
        if (lane == 0) {
            atomicAdd(&a.stats->rows_visited, c_visited);
            atomicAdd(&a.stats->rows_changed, chg_tot);
            atomicAdd(&a.stats->tasks, c_tasks);
            atomicAdd(&a.stats->rows_read, c_rows);
            atomicAdd(&a.stats->bytes_written, c_wbytes);
            atomicAdd(&a.stats->arcs_scanned, c_scanned);
            atomicAdd(&a.stats->arcs_active, c_active);
            atomicAdd(&a.stats->sectors, c_sectors);
        }
    }
}

template <bool STATS>
__global__ __launch_bounds__(kPackWG, 3) void k_propagate_pack(const PropArgs* __restrict__ args, Batch B, int maxJ, int pb)
{
    IMX_BATCH_PROLOGUE(PropArgs);
    propagate_pack_body<STATS>(a, lb, lg, maxJ, pb);
}

// Launch-configuration caches below are shared by every engine of the
// process; engines may step on different host threads.
static std::mutex g_launch_cfg_mutex;

static int cu_count()
{
    static const int cus = [] {
        int dev = 0, c = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        return c < 1 ? 1 : c;
    }();
    return cus;
}

template <int GS, int DPLG, bool STATS>
static size_t propagate_lds(int J)
{
    constexpr int NG = 64 / GS;
    return sizeof(uint32_t) * ((size_t)J + kTableWords + (size_t)kWaves * kPropBufCap +
                               (size_t)kWaves * NG * ((size_t)(J / 4) + group_buf_words<GS, STATS>()));
}

// Occupancy-derived workgroups per CU of one propagation configuration.
template <int GS, int DPLG, bool STATS>
static hipError_t propagate_setup(int J, int* per_cu)
{
    const size_t lds = propagate_lds<GS, DPLG, STATS>(J);
    std::lock_guard<std::mutex> lock(g_launch_cfg_mutex);
    static size_t lds_set = 0, attr_set = 0;
    static int cached = 0;
    if (lds_set != lds) {
        if (lds > attr_set) {
            hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_propagate<GS, DPLG, STATS>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (err != hipSuccess) return err;
            attr_set = lds;
        }
        hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&cached, k_propagate<GS, DPLG, STATS>, kWG, lds);
        if (err != hipSuccess) return err;
        if (cached < 1) cached = 1;
        lds_set = lds;
    }
    *per_cu = cached;
    return hipSuccess;
}

template <int GS, int DPLG, bool STATS>
static hipError_t launch_propagate_t(const PropArgs* args, const Batch& B, int maxJ, hipStream_t st)
{
    int per_cu = 0;
    hipError_t err = propagate_setup<GS, DPLG, STATS>(maxJ, &per_cu);
    if (err != hipSuccess) return err;
    const size_t lds = propagate_lds<GS, DPLG, STATS>(maxJ);
    hipLaunchKernelGGL((k_propagate<GS, DPLG, STATS>), dim3(B.wg0[B.nq]), dim3(kWG), lds, st, args, B);
    return hipGetLastError();
}

// Lane-group size for a row width: the smallest of 16/32/64 lanes that keeps
// at most 16 words of the row per lane, unless a larger one is requested.
// Lanes per task: the lane-group size (16, 32 or 64, at least what keeps 16
// words of the row per lane), or for the packed kernel (requested 0) the
// wave's 64 lanes shared by pack_rows(J, pack_bytes()) tasks.
int propagate_group_size(int J, int requested)
{
    if (requested == 0) {
        const int l = 64 / pack_rows(J, pack_bytes());
        return l < 1 ? 1 : l;
    }
    int gs = (J <= 1024) ? 16 : (J <= 2048) ? 32 : 64;
    if (requested == 16 || requested == 32 || requested == 64) gs = requested > gs ? requested : gs;
    return gs;
}

static size_t pack_lds(int maxJ, bool stats)
{
    return sizeof(uint32_t) * (size_t)pack_lds_words(maxJ, pack_bytes(), stats);
}

template <bool STATS>
static hipError_t pack_setup(int maxJ, int* per_cu)
{
    const size_t lds = pack_lds(maxJ, STATS);
    std::lock_guard<std::mutex> lock(g_launch_cfg_mutex);
    static size_t lds_set = 0, attr_set = 0;
    static int cached = 0;
    if (lds_set != lds) {
        if (lds > attr_set) {
            hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_propagate_pack<STATS>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (err != hipSuccess) return err;
            attr_set = lds;
        }
        hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&cached, k_propagate_pack<STATS>, kPackWG, lds);
        if (err != hipSuccess) return err;
        if (cached < 1) cached = 1;
        lds_set = lds;
    }
    *per_cu = cached;
    return hipSuccess;
}

// Calls f.template operator()<GS, DPLG, STATS>() for the configuration of
// (maxJ, gs, stats).
template <class F>
static hipError_t propagate_dispatch(int maxJ, int gs, bool stats, F&& f)
{
    const int g = propagate_group_size(maxJ, gs);
    const int dpl = (maxJ / 4 + g - 1) / g;
#define IMX_PD(G, D)                                                                         \
    if (g == G && dpl <= D) return stats ? f.template operator()<G, D, true>() : f.template operator()<G, D, false>();
    IMX_PD(16, 1) IMX_PD(16, 2) IMX_PD(16, 4) IMX_PD(16, 8) IMX_PD(16, 16)
    IMX_PD(32, 1) IMX_PD(32, 2) IMX_PD(32, 4) IMX_PD(32, 8) IMX_PD(32, 16)
    IMX_PD(64, 1) IMX_PD(64, 2) IMX_PD(64, 4) IMX_PD(64, 8) IMX_PD(64, 16)
#undef IMX_PD
    return hipErrorInvalidValue;
}

hipError_t propagate_full_grid(int maxJ, int gs, bool stats, int* grid)
{
    if (gs == 0) {
        int per_cu = 0;
        const hipError_t e = stats ? pack_setup<true>(maxJ, &per_cu) : pack_setup<false>(maxJ, &per_cu);
        *grid = cu_count() * per_cu;
        return e;
    }
    return propagate_dispatch(maxJ, gs, stats, [&]<int G, int D, bool S>() -> hipError_t {
        int per_cu = 0;
        hipError_t e = propagate_setup<G, D, S>(maxJ, &per_cu);
        *grid = cu_count() * per_cu;
        return e;
    });
}

int propagate_lanes_per_task(int maxJ, int gs) { return propagate_group_size(maxJ, gs); }

int propagate_wg_threads(int gs) { return gs == 0 ? kPackWG : kWG; }

hipError_t launch_propagate(const PropArgs* args, const Batch& B, int maxJ, int gs, bool stats, hipStream_t st)
{
    if (gs == 0) {
        int per_cu = 0;
        hipError_t e = stats ? pack_setup<true>(maxJ, &per_cu) : pack_setup<false>(maxJ, &per_cu);
        if (e != hipSuccess) return e;
        const size_t lds = pack_lds(maxJ, stats);
        const int pb = pack_bytes();
        if (stats)
            hipLaunchKernelGGL(k_propagate_pack<true>, dim3(B.wg0[B.nq]), dim3(kPackWG), lds, st, args, B, maxJ, pb);
        else
            hipLaunchKernelGGL(k_propagate_pack<false>, dim3(B.wg0[B.nq]), dim3(kPackWG), lds, st, args, B, maxJ, pb);
        return hipGetLastError();
    }
    return propagate_dispatch(maxJ, gs, stats, [&]<int G, int D, bool S>() -> hipError_t {
        return launch_propagate_t<G, D, S>(args, B, maxJ, st);
    });
}

// Before sweep s: clear the bitmap sweep s writes and the counters sweep s
// accumulates into, and compact the vertices the mark step of sweep s-1
// flagged into sweep s's active task list (unless sweep s visits every task).
// Sweep 0 (right after a fill) marks every row as changed.
__global__ __launch_bounds__(kWG) void k_sweep_prep(const PrepArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(PrepArgs);
    __shared__ int32_t wbuf[kWaves][kWaveBufCap];
    const auto& s = a.s;
    const int sweep = a.sweep;
    const int64_t i0 = lb * blockDim.x + threadIdx.x;
    if (sweep > 0 && *s.conv != ~0u) return;  // the build has converged
    if (sweep == 0 && i0 == 0) *s.conv = ~0u;   // a new build starts
    uint32_t* nxt = s.chg[(sweep + 1) & 1];
    for (int64_t i = i0; i < a.nwords; i += lg * blockDim.x) {
        nxt[i] = 0u;
        if (sweep == 0) s.chg[0][i] = 0xffffffffu;
    }
    if (i0 == 0) {
        s.rows_changed[sweep & 3] = 0ull;
        s.chg_count[sweep & 3] = 0u;
        s.act_count[(sweep + 1) & 3] = 0u;
    }
    if (sweep > 0 && s.dense[sweep & 3] == 0u && s.chg_count[(sweep - 1) & 3] != 0u) {
        __shared__ uint32_t s_flush[kWaves + 1];
        const int wave = (int)(threadIdx.x >> 6);
        WaveList L{wbuf[wave], 0, s.act_tasks[sweep & 1], &s.act_count[sweep & 3]};
        compact_flags<false>(s.act8, s.act_blk, a.n, a.task_start, L, L, nullptr, 0u, lb * kWaves + wave, lg * kWaves);
        wg_flush(L, s_flush);
    }
}

hipError_t launch_sweep_prep(const PrepArgs* args, const Batch& B, hipStream_t st)
{
    hipLaunchKernelGGL(k_sweep_prep, dim3(B.wg0[B.nq]), dim3(kWG), 0, st, args, B);
    return hipGetLastError();
}

// Mark step of sweep s: every source w of an in-arc of a changed row is
// flagged active for sweep s+1 (plain byte stores; the prep step of sweep s+1
// compacts the flags into the task list).
__global__ __launch_bounds__(kWG) void k_mark(const MarkArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(MarkArgs);
    const auto& g = a.g;
    const auto& s = a.s;
    const int sweep = a.sweep;
    const int lane = lane_id();
    // Many changed rows (more than n / dense_div): the next sweep visits every
    // task (with per-arc changed-head tests) instead of building a list.
    if (*s.conv != ~0u) return;  // converged before this sweep
    const unsigned long long changed = s.rows_changed[sweep & 3];
    if (changed == 0ull) {       // sweep s changed nothing: the build has converged at s
        if (lb == 0 && threadIdx.x == 0) *s.conv = (uint32_t)sweep;
        return;
    }
    const bool dense = changed * (unsigned long long)a.dense_div > (unsigned long long)g.n;
    if (lb == 0 && threadIdx.x == 0) s.dense[(sweep + 1) & 3] = dense ? 1u : 0u;
    if (dense) return;
    const uint32_t count = s.chg_count[sweep & 3];
    const int64_t nw = lg * kWaves;
    for (int64_t q = lb * kWaves + (threadIdx.x >> 6); q < (int64_t)count; q += nw) {
        const int32_t it = s.chg_list[q];
        const int32_t v = g.in_task_v[it];
        const int64_t e0 = g.in_task_e0[it];
        const int64_t ve = g.in_rowptr[v + 1];
        const int64_t e1 = (e0 + g.in_split < ve) ? e0 + g.in_split : ve;
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const int32_t w = g.in_col[e];
            s.act8[w] = 1u;
            s.act_blk[w >> kFlagBlockShift] = 1u;
        }
    }
}

hipError_t launch_mark(const MarkArgs* args, const Batch& B, hipStream_t st)
{
    hipLaunchKernelGGL(k_mark, dim3(B.wg0[B.nq]), dim3(kWG), 0, st, args, B);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a5: estimate terms per vertex (Eq. 7 harmonic form over uncovered registers):
// Ju = #registers != 0, Hu = sum of 2^(33 - M).  One wave per row.

// Sum of x over the aligned group of L lanes (L a power of two).
__device__ __forceinline__ uint32_t group_sum_u32(uint32_t x, int L)
{
    for (int d = L >> 1; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}
__device__ __forceinline__ unsigned long long group_sum_u64(unsigned long long x, int L)
{
    for (int d = L >> 1; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Ju and Hu terms of one 32-bit word of registers (covered registers are 0,
// uncovered ones 1..33).  Without branches: every byte adds 2^(33 - r), a
// covered one 2^33, and the caller subtracts 2^33 per covered register once
// the uncovered count c is known (Hu = h - 2^33 * (registers - c)).
__device__ __forceinline__ void est_word(uint32_t d, uint32_t& c, unsigned long long& h)
{
    // high bit of every nonzero byte
    const uint32_t nz = (((d & 0x7f7f7f7fu) + 0x7f7f7f7fu) | d) & 0x80808080u;
    c += (uint32_t)__builtin_popcount(nz);
#pragma unroll
    for (int b = 0; b < 4; ++b) h += 1ull << (33u - ((d >> (8 * b)) & 0xffu));
}

__global__ __launch_bounds__(kWG) void k_estimate(const EstArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(EstArgs);
    if (a.am_dirty != nullptr && lb == 0)  // every estimate term is recomputed
        for (int i = threadIdx.x; i < kArgmaxBlocks; i += blockDim.x) a.am_dirty[i] = 1u;
    const int L = row_lanes(a.J);
    const int lane = lane_id();
    const int sub = lane % L;
    const int chunks = a.J / 16;
    const int64_t rpw = 64 / L;  // rows of a wave per batch slot
    const int64_t per_wave = rpw * kRowBatch;
    const int64_t nw = lg * kWaves;
    const uint4* M4 = reinterpret_cast<const uint4*>(a.M);
    // every lane of a wave runs the same number of iterations (uniform shuffles)
    for (int64_t vb = (lb * kWaves + (threadIdx.x >> 6)) * per_wave; vb < a.n; vb += nw * per_wave) {
        uint32_t c[kRowBatch];
        unsigned long long h[kRowBatch];
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r) {
            c[r] = 0;
            h[r] = 0;
        }
        for (int k = sub; k < chunks; k += L) {
            uint4 q[kRowBatch];
#pragma unroll
            for (int r = 0; r < kRowBatch; ++r) {
                const int64_t v = vb + r * rpw + lane / L;
                q[r] = (v < a.n) ? M4[(size_t)v * (size_t)chunks + k] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int r = 0; r < kRowBatch; ++r) {
                est_word(q[r].x, c[r], h[r]);
                est_word(q[r].y, c[r], h[r]);
                est_word(q[r].z, c[r], h[r]);
                est_word(q[r].w, c[r], h[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r) {
            const int64_t v = vb + r * rpw + lane / L;
            const uint32_t cs = group_sum_u32(c[r], L);
            const unsigned long long hs = group_sum_u64(h[r], L);
            if (sub == 0 && v < a.n) {
                a.Ju[v] = cs;
                a.Hu[v] = hs - ((unsigned long long)((uint32_t)a.J - cs) << 33);  // drop covered registers' 2^33
            }
        }
    }
}

hipError_t launch_estimate(const EstArgs* args, const Batch& B, hipStream_t st)
{
    hipLaunchKernelGGL(k_estimate, dim3(B.wg0[B.nq]), dim3(kWG), 0, st, args, B);
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

// Partial b (0 <= b < nparts) covers the vertices v with (v / 256) % nparts
// == b.  Workgroup lb of the query's lg computes partials lb, lb + lg, ..., so
// every one of the nparts slots the final pass reads is written whatever the
// grid (a capped grid gives fewer workgroups than partials).
__global__ __launch_bounds__(256) void k_argmax_partial(const ArgmaxArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(ArgmaxArgs);
    for (int64_t b = lb; b < a.nparts; b += lg) {
        if (a.am.dirty != nullptr && a.am.dirty[b] == 0u) continue;  // unchanged since computed (uniform)
        Cand best{0u, 0ull, -1};
        for (int64_t v = b * blockDim.x + threadIdx.x; v < a.n; v += (int64_t)a.nparts * blockDim.x) {
            if (a.is_seed[v]) continue;
            Cand c{a.Ju[v], a.Hu[v], (int32_t)v};
            if (better(c, best)) best = c;
        }
        block_reduce_best(best);
        if (threadIdx.x == 0) {
            a.am.pJ[b] = best.J;
            a.am.pH[b] = best.H;
            a.am.pid[b] = best.id;
            if (a.am.dirty != nullptr) a.am.dirty[b] = 0u;
        }
        __syncthreads();  // block_reduce_best's LDS is reused by the next partial
    }
}

// One workgroup per query reduces that query's a.nparts partial winners.
__global__ __launch_bounds__(256) void k_argmax_final(const ArgmaxArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(ArgmaxArgs);
    Cand best{0u, 0ull, -1};
    for (int i = threadIdx.x; i < a.nparts; i += blockDim.x) {
        Cand c{a.am.pJ[i], a.am.pH[i], a.am.pid[i]};
        if (better(c, best)) best = c;
    }
    block_reduce_best(best);
    if (threadIdx.x == 0) *a.best = best.id;
}

hipError_t launch_argmax(const ArgmaxArgs* args, const Batch& partial, const Batch& final_, hipStream_t st)
{
    hipLaunchKernelGGL(k_argmax_partial, dim3(partial.wg0[partial.nq]), dim3(256), 0, st, args, partial);
    hipLaunchKernelGGL(k_argmax_final, dim3(final_.wg0[final_.nq]), dim3(256), 0, st, args, final_);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a7: covering cascade (Alg. 3), union-frontier BFS over all simulations.
// Frontier lists hold out-tasks, so a hub's arcs are spread over many waves.

__device__ __forceinline__ uint32_t marker(int t) { return 64u + ((uint32_t)t & 63u); }
__device__ __forceinline__ bool uncovered(uint32_t b) { return b >= 1u && b <= 33u; }

// Level 0: the pick s becomes a seed and is covered in every simulation where
// it is not yet covered; its out-tasks form frontier Q_1.
__global__ __launch_bounds__(64) void k_cascade_seed(const SeedArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(SeedArgs);
    const auto& g = a.g;
    const auto& c = a.c;
    const int lane = lane_id();
    const int32_t s = *a.best;
    if (s < 0 || (int64_t)s >= g.n) {  // no candidate (cannot happen for K <= n); leave an empty cascade
        if (lane == 0) {
            a.seeds[a.k] = -1;
            c.qsize[0] = c.qsize[1] = c.qsize[2] = c.qsize[3] = 0;
            *c.ntouched = 0;
            *c.level_end = ~0u;
        }
        return;
    }
    uint32_t* row = reinterpret_cast<uint32_t*>(a.M + (size_t)s * (size_t)a.J);
    bool any = false;
    const uint32_t mk = marker(0);
    for (int idx = lane; idx < (a.J >> 2); idx += 64) {
        const uint32_t d = row[idx];
        const uint32_t um = uncovered_mask4(d);
        if (um) {
            row[idx] = (d & ~um) | ((mk * 0x01010101u) & um);
            any = true;
        }
    }
    const bool anyw = __ballot(any) != 0ull;
    const int32_t t0 = g.task_start[s], nt = anyw ? g.task_start[s + 1] - t0 : 0;
    for (int q = lane; q < nt; q += 64) c.q[1][q] = t0 + q;
    if (lane == 0) {
        a.is_seed[s] = 1;
        a.seeds[a.k] = s;
        a.pickJ[a.k] = a.Ju[s];
        a.pickH[a.k] = a.Hu[s];
        c.qsize[0] = 0;
        c.qsize[2] = 0;
        c.qsize[3] = 0;
        c.qsize[1] = (uint32_t)nt;
        *c.level_end = ~0u;
        c.touched[0] = s;
        *c.ntouched = 1;
        c.touch_stamp[s] = a.cascade_id;
    }
}

hipError_t launch_cascade_seed(const SeedArgs* args, const Batch& B, hipStream_t st)
{
    hipLaunchKernelGGL(k_cascade_seed, dim3(B.wg0[B.nq]), dim3(64), 0, st, args, B);
    return hipGetLastError();
}

// Level t >= 1: each task of Q_t expands its vertex u along its arcs, in the
// simulations where u was covered at level t-1 (registers holding the level
// t-1 marker).  Those simulations are listed as the 32-bit words of u's row
// that contain the marker (ED, ascending); each arc's candidate range selects
// a contiguous slice of ED, and the (arc, word) items are dealt to lanes.
// Heads still uncovered where the arc is live get the level-t marker (byte
// stores) and are flagged in lv8; the compaction after the level turns the
// flags into Q_{t+1}.

constexpr int kLevelBufWords = 5 * 64;

__device__ __forceinline__ int lower_bound_i32(const int* A, int n, int key)
{
    int lo = 0, len = n;
    while (len > 0) {
        const int half = len >> 1;
        if (A[lo + half] < key) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// Set of vertex ids in LDS for one workgroup (open addressing, linear
// probing, LDS atomics only): the tail kernels collect the distinct vertices
// of the next frontier in it.  Slots hold id + 1 (0: empty); the distinct ids
// are listed in insertion order.  Once `cap` ids are listed, further new ids
// are not taken and the caller handles them itself (overflow).
struct LdsSet {
    uint32_t* slots;     // H words
    int32_t* list;       // cap entries
    uint32_t* count;     // distinct ids seen (may exceed cap on overflow)
    uint32_t* overflow;  // nonzero once an id could not be listed
    int H;               // a power of two, at least 2 * cap
    int cap;
};

// Clears the set (every thread of the workgroup calls it; a barrier follows).
__device__ __forceinline__ void lds_set_clear(LdsSet& S)
{
    for (int i = threadIdx.x; i < S.H; i += blockDim.x) S.slots[i] = 0u;
    if (threadIdx.x == 0) {
        *S.count = 0u;
        *S.overflow = 0u;
    }
}

// Adds v; false when v is new but the list is full (the caller keeps v by
// other means), true otherwise (listed now or before).
__device__ __forceinline__ bool lds_set_insert(LdsSet& S, int32_t v)
{
    const uint32_t key = (uint32_t)v + 1u;
    uint32_t h = (key * 2654435761u) & (uint32_t)(S.H - 1);
    for (int probe = 0; probe < S.H; ++probe) {
        const uint32_t cur = S.slots[h];
        if (cur == key) return true;
        if (cur == 0u) {
            if (__atomic_load_n(S.count, __ATOMIC_RELAXED) >= (uint32_t)S.cap) break;
            const uint32_t prev = atomicCAS(&S.slots[h], 0u, key);
            if (prev == 0u) {
                const uint32_t pos = atomicAdd(S.count, 1u);
                if (pos < (uint32_t)S.cap) {
                    S.list[pos] = v;
                    return true;
                }
                break;
            }
            if (prev == key) return true;
        }
        h = (h + 1u) & (uint32_t)(S.H - 1);
    }
    atomicOr(S.overflow, 1u);
    return false;
}

// The body works for workgroup lb of lg workgroups assigned to one query.
// TAIL (the single-workgroup tail kernel): newly covered heads go into the
// LDS set S instead of the flag array (into the flags only when S is full).
// NW: waves per workgroup (the per-wave LDS areas follow the table).
template <bool TAIL, int NW = kWaves>
__device__ __forceinline__ void cascade_level_body(const LevelArgsT<true>& a, int64_t lb, int64_t lg, LdsSet* S)
{
    extern __shared__ uint32_t smem[];
    const int J = a.J;
    const int Jw = J >> 2;
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = lane_id();

    const uint32_t qn = a.c.qsize[a.t & 3];
    if (lb == 0 && threadIdx.x == 0) {
        a.c.qsize[(a.t + 1) & 3] = 0;  // Q_{t+1}, filled by the compaction
        if (qn == 0u && *a.c.level_end == ~0u) *a.c.level_end = (uint32_t)a.t;
    }
    if (lb * NW >= (int64_t)qn) return;  // no task for this workgroup (uniform)

    uint32_t* sX = smem;
    const uint32_t* sT = smem + J;
    const int XT = J + kTableWords;
    uint32_t* roww = smem + XT + wave * (2 * Jw + kLevelBufWords);
    int* ED = reinterpret_cast<int*>(roww + Jw);
    int* ev = ED + Jw;
    uint32_t* eh = reinterpret_cast<uint32_t*>(ev + 64);
    uint32_t* eW = eh + 64;
    int* epl = reinterpret_cast<int*>(eW + 64);
    int* est = epl + 64;

    for (int i = threadIdx.x; i < J + kBuckets + 1; i += 64 * NW) sX[i] = a.X[i];
    __syncthreads();

    const int32_t* Q = (a.t & 1) ? a.c.q[1] : a.c.q[0];  // a select, not an index: keeps a local record in registers
    uint8_t* lv8 = a.c.lv8;
    const uint32_t mk_prev = marker(a.t - 1);
    const uint32_t mk_cur = marker(a.t);
    const auto& g = a.g;
    const uint32_t* M32 = reinterpret_cast<const uint32_t*>(a.M);
    const int64_t nw = lg * NW;

    // Task records are loaded one task ahead and task ids two ahead; the
    // first chunk of arcs is loaded with u's row, and every later chunk while
    // the previous one is processed.
    int64_t i = lb * NW + wave;
    int32_t t_nx = (i < (int64_t)qn) ? Q[i] : -1;
    int32_t u_nx = 0;
    int64_t e0_nx = 0;
    uint32_t len_nx = 0;
    if (t_nx >= 0) {
        u_nx = g.task_u[t_nx];
        e0_nx = g.task_e0[t_nx];
        len_nx = g.task_len[t_nx];
    }
    int32_t t_nx2 = (i + nw < (int64_t)qn) ? Q[i + nw] : -1;
    for (; i < (int64_t)qn; i += nw) {
        const int32_t u = u_nx;
        const int64_t e0 = e0_nx;
        const int64_t e1 = e0 + (int64_t)(len_nx & 0x7fffffffu);
        // the next task's records, and the id of the one after
        t_nx = t_nx2;
        if (t_nx >= 0) {
            u_nx = g.task_u[t_nx];
            e0_nx = g.task_e0[t_nx];
            len_nx = g.task_len[t_nx];
        }
        t_nx2 = (i + 2 * nw < (int64_t)qn) ? Q[i + 2 * nw] : -1;
        const uint32_t* Mu = M32 + (size_t)u * (size_t)Jw;
        int32_t v_nx = 0;
        uint32_t w_nx = 0;
        if (e0 + lane < e1) {
            v_nx = g.col[e0 + lane];
            w_nx = g.W[e0 + lane];
        }
        // u's row in 16-byte chunks (4 words per lane; Jw is a multiple of
        // 16), so a row of up to 1 KB is one load per lane
        int nE = 0;
        const uint4* Mu4 = reinterpret_cast<const uint4*>(Mu);
        for (int base = 0; base < Jw; base += 256) {
            const int w0 = base + 4 * lane;
            uint4 d = make_uint4(0u, 0u, 0u, 0u);
            if (w0 < Jw) {
                d = Mu4[w0 >> 2];
                *reinterpret_cast<uint4*>(&roww[w0]) = d;
            }
            const uint32_t hm = (eq_mask4(d.x, mk_prev) ? 1u : 0u) | (eq_mask4(d.y, mk_prev) ? 2u : 0u) |
                                (eq_mask4(d.z, mk_prev) ? 4u : 0u) | (eq_mask4(d.w, mk_prev) ? 8u : 0u);
            const int cnt = (w0 < Jw) ? __builtin_popcount(hm) : 0;
            const int incl = wave_incl_scan(cnt);
            int pos = nE + incl - cnt;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if ((hm >> k) & 1u) ED[pos++] = w0 + k;
            nE += lane_val(incl, 63);
        }
        wave_lds_sync();
        if (nE == 0) continue;
        for (int64_t cb = e0; cb < e1; cb += 64) {
            const int64_t e = cb + lane;
            int cnt = 0, pl = 0;
            const int32_t v = v_nx;
            const uint32_t w = w_nx;
            uint32_t h = 0;
            if (cb + 64 < e1) {
                v_nx = 0;
                w_nx = 0;
                if (e + 64 < e1) {
                    v_nx = g.col[e + 64];
                    w_nx = g.W[e + 64];
                }
            }
            if (e < e1) {
                h = arc_hash((uint32_t)u, (uint32_t)v);
                int lo, hi;
                candidate_range(sX, sT, J, h, w, lo, hi);
                if (hi > lo) {
                    pl = lower_bound_i32(ED, nE, lo >> 2);
                    cnt = lower_bound_i32(ED, nE, ((hi - 1) >> 2) + 1) - pl;
                }
            }
            const int incl = wave_incl_scan(cnt);
            const int total = lane_val(incl, 63);
            if (total == 0) continue;
            ev[lane] = v;
            eh[lane] = h;
            eW[lane] = w;
            epl[lane] = pl;
            est[lane] = incl - cnt;
            wave_lds_sync();
            for (int r = 0; r < total; r += 64) {
                const int idx = r + lane;
                if (idx < total) {
                    const int k = owner_of(est, idx);
                    const int d = ED[epl[k] + (idx - est[k])];
                    uint32_t m = eq_mask4(roww[d], mk_prev) &
                                 live_mask4(*reinterpret_cast<const uint4*>(&sX[4 * d]), eh[k], eW[k]);
                    if (m) {
                        const int32_t vk = ev[k];
                        const size_t off = (size_t)vk * (size_t)Jw + (size_t)d;
                        m &= uncovered_mask4(M32[off]);
                        if (m) {
                            uint8_t* p = a.M + off * 4;
#pragma unroll
                            for (int b = 0; b < 4; ++b)
                                if ((m >> (8 * b)) & 1u) p[b] = (uint8_t)mk_cur;
                            if (!TAIL || !lds_set_insert(*S, vk)) {
                                lv8[vk] = 1u;
                                a.c.lv_blk[vk >> kFlagBlockShift] = 1u;
                            }
                        }
                    }
                }
            }
            wave_lds_sync();
        }
    }
}

__global__ __launch_bounds__(kWG) void k_cascade_level(const LevelArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(LevelArgs);
    cascade_level_body<false>(a, lb, lg, nullptr);
}

__host__ __device__ static size_t level_lds(int J, int nw = kWaves)
{
    return sizeof(uint32_t) * ((size_t)J + kTableWords + (size_t)nw * ((size_t)(J / 2) + kLevelBufWords));
}

hipError_t cascade_level_full_grid(int maxJ, int* grid)
{
    std::lock_guard<std::mutex> lock(g_launch_cfg_mutex);
    static size_t lds_set = 0, attr_set = 0;
    static int per_cu = 0;
    const size_t lds = level_lds(maxJ);
    if (lds_set != lds) {
        if (lds > attr_set) {
            hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cascade_level),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (err != hipSuccess) return err;
            attr_set = lds;
        }
        hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cascade_level, kWG, lds);
        if (err != hipSuccess) return err;
        if (per_cu < 1) per_cu = 1;
        lds_set = lds;
    }
    *grid = cu_count() * per_cu;
    return hipSuccess;
}

hipError_t launch_cascade_level(const LevelArgs* args, const Batch& B, int maxJ, hipStream_t st)
{
    int grid = 0;
    hipError_t err = cascade_level_full_grid(maxJ, &grid);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_cascade_level, dim3(B.wg0[B.nq]), dim3(kWG), level_lds(maxJ), st, args, B);
    return hipGetLastError();
}

// After level t: the flagged vertices become frontier Q_{t+1} (their
// out-tasks) and join the touched list once per cascade.
__global__ __launch_bounds__(kWG) void k_cascade_compact(const LevelCompactArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(LevelCompactArgs);
    __shared__ int32_t wbuf[kWaves][2 * kWaveBufCap];
    const auto& c = a.c;
    if (c.qsize[a.t & 3] == 0u) return;  // empty level: nothing was flagged
    const int wave = (int)(threadIdx.x >> 6);
    WaveList L{wbuf[wave], 0, c.q[(a.t + 1) & 1], &c.qsize[(a.t + 1) & 3]};
    WaveList T{wbuf[wave] + kWaveBufCap, 0, c.touched, c.ntouched};
    __shared__ uint32_t s_flush[kWaves + 1];
    compact_flags<true>(c.lv8, c.lv_blk, a.n, a.task_start, L, T, c.touch_stamp, a.cascade_id, lb * kWaves + wave,
                        lg * kWaves);
    wg_flush(L, s_flush);
    wg_flush(T, s_flush);
}

hipError_t launch_cascade_compact(const LevelCompactArgs* args, const Batch& B, hipStream_t st)
{
    hipLaunchKernelGGL(k_cascade_compact, dim3(B.wg0[B.nq]), dim3(kWG), 0, st, args, B);
    return hipGetLastError();
}

// End of a cascade: markers become 0 in every touched row; Ju/Hu of touched
// rows are recomputed and T grows by the number of newly covered registers.
// Clears the cascade markers (>= 64) of one word and adds its uncovered
// registers to (c, h).
__device__ __forceinline__ uint32_t fin_word(uint32_t d, uint32_t& c, unsigned long long& h)
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t r = (d >> (8 * b)) & 0xffu;
        if (r >= 64u) {
            d &= ~(0xffu << (8 * b));
        } else if (r) {
            ++c;
            h += 1ull << (33u - r);
        }
    }
    return d;
}

__global__ __launch_bounds__(kWG) void k_cascade_finalize(const FinArgs* __restrict__ args, Batch B)
{
    IMX_BATCH_PROLOGUE(FinArgs);
    __shared__ unsigned long long s_sum[kWaves];
    const auto& c = a.c;
    if (*c.level_end == ~0u) return;  // the cascade is still running (uniform)
    const int L = row_lanes(a.J);
    const int lane = lane_id();
    const int sub = lane % L;
    const int chunks = a.J / 16;
    const int64_t rpw = 64 / L;
    const int64_t per_wave = rpw * kRowBatch;
    const int64_t nw = lg * kWaves;
    const int64_t nt = (int64_t)*c.ntouched;
    uint4* M4 = reinterpret_cast<uint4*>(a.M);
    unsigned long long dT = 0;
    for (int64_t vb = (lb * kWaves + (threadIdx.x >> 6)) * per_wave; vb < nt; vb += nw * per_wave) {
        int32_t vv[kRowBatch];
        uint32_t cn[kRowBatch];
        unsigned long long h[kRowBatch];
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r) {
            const int64_t i = vb + r * rpw + lane / L;
            vv[r] = (i < nt) ? c.touched[i] : -1;
            cn[r] = 0;
            h[r] = 0;
        }
        for (int k = sub; k < chunks; k += L) {
            uint4 q[kRowBatch];
#pragma unroll
            for (int r = 0; r < kRowBatch; ++r)
                q[r] = (vv[r] >= 0) ? M4[(size_t)vv[r] * (size_t)chunks + k] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
            for (int r = 0; r < kRowBatch; ++r) {
                if (vv[r] < 0) continue;
                const uint4 o = q[r];
                const uint4 nq = make_uint4(fin_word(o.x, cn[r], h[r]), fin_word(o.y, cn[r], h[r]),
                                            fin_word(o.z, cn[r], h[r]), fin_word(o.w, cn[r], h[r]));
                if (nq.x != o.x || nq.y != o.y || nq.z != o.z || nq.w != o.w)
                    M4[(size_t)vv[r] * (size_t)chunks + k] = nq;
            }
        }
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r) {
            const uint32_t cs = group_sum_u32(cn[r], L);
            const unsigned long long hs = group_sum_u64(h[r], L);
            if (sub == 0 && vv[r] >= 0) {
                const uint32_t old = a.Ju[vv[r]];
                a.Ju[vv[r]] = cs;
                a.Hu[vv[r]] = hs;
                dT += (unsigned long long)(old - cs);
                if (a.am_dirty != nullptr && a.nparts > 0)
                    a.am_dirty[((uint32_t)vv[r] >> 8) % (uint32_t)a.nparts] = 1u;
            }
        }
    }
    wg_add_u64(dT, c.T, s_sum);
}

hipError_t launch_cascade_finalize(const FinArgs* args, const Batch& B, hipStream_t st)
{
    hipLaunchKernelGGL(k_cascade_finalize, dim3(B.wg0[B.nq]), dim3(kWG), 0, st, args, B);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tail kernels (one workgroup per query): sweeps or cascade levels of small
// frontiers in a loop.  Between steps, registers merged by compare-and-swap
// and changed-bitmap words set by atomics are read by plain loads of other
// waves; the agent-scope acquire after each barrier invalidates the vector
// L1 so that those loads see them.

__device__ __forceinline__ void tail_barrier()
{
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ uint32_t ld_u32(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_u64(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// In-arc range [e0, e1) of in-task it.
__device__ __forceinline__ void in_task_range(const GraphDevT<true>& g, int32_t it, int64_t& e0, int64_t& e1)
{
    const int32_t v = g.in_task_v[it];
    e0 = g.in_task_e0[it];
    const int64_t ve = g.in_rowptr[v + 1];
    e1 = (e0 + g.in_split < ve) ? e0 + g.in_split : ve;
}

// Sweeps s0, s0+1, ... of one query (Alg. 2), each: propagate over the task
// list, then (in place of the mark and prep steps) the distinct sources of
// the in-arcs of the changed rows, collected in the LDS set, give the next
// list.  Stops when a sweep changes nothing (converged), when the next sweep
// must visit every task, when the changed rows have more than arcs_max
// in-arcs (their sources are then flagged as the mark step does), when the
// next list has more than tasks_max tasks, or after `rounds` sweeps; *next
// is the sweep the full-grid path runs next (its prep step finds the list,
// the flags or the dense switch as after its own mark step).
__global__ __launch_bounds__(kPackWG, 1) void k_tail_sweeps(const TailSweepArgs* __restrict__ args, Batch B, int maxJ,
                                                            int pb)
{
    IMX_BATCH_PROLOGUE(TailSweepArgs);
    if (lb != 0) return;
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_cnt, s_ovf, s_pos;
    __shared__ unsigned long long s_arcs;
    uint32_t* tl = smem + pack_lds_words(maxJ, pb, false);
    LdsSet S{tl, reinterpret_cast<int32_t*>(tl + kTailSlots), &s_cnt, &s_ovf, kTailSlots, kTailCap};
    const auto& g = a.g;
    const auto& sw = a.s;
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    uint32_t next = (uint32_t)(a.s0 + a.rounds), why = kTailStopRounds;
    int s = a.s0;
    if ((int64_t)ld_u32(&sw.act_count[s & 3]) > a.tasks_max) {  // the first list is too long: hand back at once
        if (threadIdx.x == 0) {
            *a.next = (uint32_t)s;
            *a.reason = kTailStopLarge;
        }
        return;
    }
    for (int i = 0; i < a.rounds; ++i, ++s) {
        // in-tasks of the rows changed in sweep s-1 (i = 0: the full-grid
        // sweep s0-1) and of those changed in sweep s
        const auto list_in = (i & 1) ? a.chg_list2 : sw.chg_list;
        const auto list_out = (i & 1) ? sw.chg_list : a.chg_list2;
        const PropArgsT<true> pa{g,        a.X,      a.J,           a.M,
                                 sw.act_tasks[s & 1], &sw.act_count[s & 3], sw.chg[s & 1], sw.chg[(s + 1) & 1],
                                 list_out, &sw.chg_count[s & 3], &sw.dense[s & 3], sw.conv,
                                 &sw.rows_changed[s & 3], nullptr, nullptr, 0u};
        propagate_pack_body<false>(pa, 0, 1, maxJ, pb);
        tail_barrier();
        const unsigned long long changed = ld_u64(&sw.rows_changed[s & 3]);
        if (changed == 0ull) {  // converged at sweep s
            if (threadIdx.x == 0) *sw.conv = (uint32_t)s;
            next = (uint32_t)s + 1u;
            why = kTailStopDone;
            break;
        }
        const bool dense = changed * (unsigned long long)a.dense_div > (unsigned long long)g.n;
        if (threadIdx.x == 0) {
            sw.dense[(s + 1) & 3] = dense ? 1u : 0u;
            sw.act_count[(s + 1) & 3] = 0u;
            s_arcs = 0ull;
            s_pos = 0u;
        }
        if (dense) {
            next = (uint32_t)s + 1u;
            why = kTailStopLarge;
            break;
        }
        const uint32_t nin = ld_u32(&sw.chg_count[s & 3]);
        lds_set_clear(S);
        __syncthreads();
        // in-arcs of the changed rows
        unsigned long long na = 0;
        for (uint32_t q = threadIdx.x; q < nin; q += blockDim.x) {
            int64_t e0, e1;
            in_task_range(g, list_out[q], e0, e1);
            na += (unsigned long long)(e1 - e0);
        }
        na = wave_sum_u64(na);
        if (lane == 0 && na) atomicAdd(&s_arcs, na);
        __syncthreads();
        const bool flag = s_arcs > (unsigned long long)a.arcs_max;
        for (uint32_t q = wave; q < nin; q += kPackWaves) {
            int64_t e0, e1;
            in_task_range(g, list_out[q], e0, e1);
            for (int64_t e = e0 + lane; e < e1; e += 64) {
                const int32_t w = g.in_col[e];
                if (flag || !lds_set_insert(S, w)) {
                    sw.act8[w] = 1u;
                    sw.act_blk[w >> kFlagBlockShift] = 1u;
                }
            }
        }
        __syncthreads();
        if (flag || s_ovf) {  // the prep step of sweep s+1 compacts the flags
            for (uint32_t k = threadIdx.x; k < min(s_cnt, (uint32_t)kTailCap); k += blockDim.x) {
                sw.act8[S.list[k]] = 1u;
                sw.act_blk[S.list[k] >> kFlagBlockShift] = 1u;
            }
            next = (uint32_t)s + 1u;
            why = kTailStopLarge;
            break;
        }
        // the list of sweep s+1: the out-tasks of the distinct sources
        const auto out = sw.act_tasks[(s + 1) & 1];
        for (uint32_t k = threadIdx.x; k < s_cnt; k += blockDim.x) {
            const int32_t w = S.list[k];
            const int32_t t0 = g.task_start[w], cnt = g.task_start[w + 1] - t0;
            const uint32_t pos = atomicAdd(&s_pos, (uint32_t)cnt);
            for (int q = 0; q < cnt; ++q) out[pos + q] = t0 + q;
        }
        // clear the changed bits of sweep s-1 (read by this sweep) for reuse by
        // sweep s+1: the rows with in-arcs are those of list_in; bits of rows
        // without in-arcs are never read and only ever set again
        const uint32_t nprev = ld_u32(&sw.chg_count[(s - 1) & 3]);
        for (uint32_t q = threadIdx.x; q < nprev; q += blockDim.x) {
            const int32_t v = g.in_task_v[list_in[q]];
            sw.chg[s & 1][(uint32_t)v >> 5] = 0u;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            sw.act_count[(s + 1) & 3] = s_pos;
            sw.rows_changed[(s + 1) & 3] = 0ull;
            sw.chg_count[(s + 1) & 3] = 0u;
        }
        const bool stop = (int64_t)s_pos > a.tasks_max;
        tail_barrier();
        if (stop) {
            next = (uint32_t)s + 1u;
            why = kTailStopLarge;
            break;
        }
    }
    if (threadIdx.x == 0) {
        *a.next = next;
        *a.reason = why;
    }
}

// Levels t0, t0+1, ... of one cascade (Alg. 3): each expands Q_t; the
// distinct newly covered heads, collected in the LDS set, give Q_{t+1} (their
// out-tasks) and join the touched list once per cascade.  Stops at an empty
// frontier (the cascade is over: level_end), before a frontier of more than
// tasks_max tasks, when the LDS set fills up (the heads of level t are then
// flagged and *cmp_pending = t: the compaction of level t must run before
// level t+1), or after `rounds` levels; *next is the level the full-grid
// path runs next.
constexpr int kTailLevelWaves = 8;

__global__ __launch_bounds__(64 * kTailLevelWaves, 1) void k_tail_levels(const TailLevelArgs* __restrict__ args, Batch B,
                                                                         int maxJ)
{
    IMX_BATCH_PROLOGUE(TailLevelArgs);
    if (lb != 0) return;
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_cnt, s_ovf, s_pos, s_tpos;
    uint32_t* tl = smem + level_lds(maxJ, kTailLevelWaves) / sizeof(uint32_t);
    LdsSet S{tl, reinterpret_cast<int32_t*>(tl + kTailSlots), &s_cnt, &s_ovf, kTailSlots, kTailCap};
    const auto& g = a.g;
    const auto& c = a.c;
    uint32_t next = (uint32_t)(a.t0 + a.rounds), pending = ~0u, why = kTailStopRounds;
    int t = a.t0;
    for (int i = 0; i < a.rounds; ++i, ++t) {
        const uint32_t qn = ld_u32(&c.qsize[t & 3]);
        if (qn == 0u) {  // empty frontier: the cascade ended at level t
            if (threadIdx.x == 0 && *c.level_end == ~0u) *c.level_end = (uint32_t)t;
            next = (uint32_t)t;
            why = kTailStopDone;
            break;
        }
        if (qn > a.tasks_max) {
            next = (uint32_t)t;
            why = kTailStopLarge;
            break;
        }
        lds_set_clear(S);
        if (threadIdx.x == 0) {
            s_pos = 0u;
            s_tpos = 0u;
        }
        __syncthreads();
        const LevelArgsT<true> la{g, a.X, a.J, a.M, c, t};
        cascade_level_body<true, kTailLevelWaves>(la, 0, 1, &S);
        tail_barrier();
        if (s_ovf) {  // heads beyond the set were flagged; flag the listed ones too
            for (uint32_t k = threadIdx.x; k < min(s_cnt, (uint32_t)kTailCap); k += blockDim.x) {
                c.lv8[S.list[k]] = 1u;
                c.lv_blk[S.list[k] >> kFlagBlockShift] = 1u;
            }
            pending = (uint32_t)t;
            next = (uint32_t)t + 1u;
            why = kTailStopLarge;
            break;
        }
        const uint32_t base_t = ld_u32(c.ntouched);
        const auto out = ((t + 1) & 1) ? c.q[1] : c.q[0];
        for (uint32_t k = threadIdx.x; k < s_cnt; k += blockDim.x) {
            const int32_t v = S.list[k];
            const int32_t t0 = g.task_start[v], cnt = g.task_start[v + 1] - t0;
            const uint32_t pos = atomicAdd(&s_pos, (uint32_t)cnt);
            for (int q = 0; q < cnt; ++q) out[pos + q] = t0 + q;
            if (c.touch_stamp[v] != a.cascade_id) {
                c.touch_stamp[v] = a.cascade_id;
                c.touched[base_t + atomicAdd(&s_tpos, 1u)] = v;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            c.qsize[(t + 1) & 3] = s_pos;
            *c.ntouched = base_t + s_tpos;
        }
        tail_barrier();
    }
    if (threadIdx.x == 0) {
        *a.next = next;
        *a.cmp_pending = pending;
        *a.reason = why;
    }
}

template <class K>
static hipError_t tail_setup(K kernel, size_t lds, size_t* attr_set)
{
    std::lock_guard<std::mutex> lock(g_launch_cfg_mutex);
    if (lds > *attr_set) {
        hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (err != hipSuccess) return err;
        *attr_set = lds;
    }
    return hipSuccess;
}

hipError_t launch_tail_sweeps(const TailSweepArgs* args, const Batch& B, int maxJ, hipStream_t st)
{
    static size_t attr_set = 0;
    const int pb = pack_bytes();
    const size_t lds = sizeof(uint32_t) * ((size_t)pack_lds_words(maxJ, pb, false) + kTailSlots + kTailCap);
    hipError_t err = tail_setup(&k_tail_sweeps, lds, &attr_set);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_tail_sweeps, dim3(B.wg0[B.nq]), dim3(kPackWG), lds, st, args, B, maxJ, pb);
    return hipGetLastError();
}

hipError_t launch_tail_levels(const TailLevelArgs* args, const Batch& B, int maxJ, hipStream_t st)
{
    static size_t attr_set = 0;
    const size_t lds = level_lds(maxJ, kTailLevelWaves) + sizeof(uint32_t) * ((size_t)kTailSlots + kTailCap);
    hipError_t err = tail_setup(&k_tail_levels, lds, &attr_set);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_tail_levels, dim3(B.wg0[B.nq]), dim3(64 * kTailLevelWaves), lds, st, args, B, maxJ);
    return hipGetLastError();
}

int device_cu_count() { return cu_count(); }

}  // namespace imx
