// Query engine: runs any number of influence-maximisation queries (graph, J,
// seed, K) to completion together.  Every query follows Alg. 4 on one device
// (build, then K x [estimate, argmax, cascade, score, rebuild test]); the
// engine advances all active queries one stage per tick and issues one
// batched launch per kernel kind per tick, so small queries share launches and
// a single host synchronisation.  Each query's results are independent of the
// others in the mix: the fixed point, the cascade and the exact argmax do not
// depend on scheduling.
//
// Also implements the C ABI of sketches (one-query engines), engines and the
// batch entry point.
#include "handles.h"

#include <chrono>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>

namespace imx {
namespace {

// Sweeps / cascade levels per tick at most.  Convergence and the end of a
// cascade are detected on the device; launches past them return at once.
constexpr int kMaxRounds = 16;
// Partial-argmax workgroups per query in graph mode.
constexpr int kGraphArgmaxBlocks = 32;

// Per-query counters the host reads back every tick (one array per engine).
struct SlotStatus {
    unsigned long long rows_changed[4];
    unsigned long long T;
    uint32_t qsize[4];
    uint32_t act_count[4];
    uint32_t chg_count[4];
    uint32_t dense[4];
    uint32_t ntouched;
    uint32_t conv;       // first sweep of the build that changed nothing (~0u: none yet)
    uint32_t level_end;  // first empty level of the cascade (~0u: running)
    uint32_t tail_next;  // after a tail-sweeps launch: the sweep the full-grid path runs next
    uint32_t lv_next;    // after a tail-levels launch: the level the full-grid path runs next
    uint32_t cmp_pending;  // after a tail-levels launch: level whose flags await compaction (~0u: none)
    uint32_t tail_reason;  // why the last tail launch stopped (kTailStop*)
    uint32_t pad[15];
};
static_assert(sizeof(SlotStatus) == 192, "status record size");


// Paused: stopped before pick `pause_k` with current registers and estimate
// terms (the parity hook im_select_seeds_until).
enum class Stage { Fill, Sweeps, Estimate, Pick, Levels, Built, Paused, Done, Failed };

}  // namespace

double estimate_value(int J, uint32_t Ju, unsigned long long Hu)
{
    if (Ju == 0) return 0.0;
    const double alpha = (J == 16) ? 0.673 : (J == 32) ? 0.697 : (J == 64) ? 0.709 : 0.7213 / (1.0 + 1.079 / (double)J);
    const volatile double scale = alpha * 8589934592.0;
    const volatile double num = (double)((uint64_t)Ju * Ju);
    const volatile double den = (double)J * (double)Hu;
    const volatile double qv = num / den;
    return scale * qv;
}

namespace {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct Query {
    int64_t id = 0;
    int slot = -1;
    const im_graph* g = nullptr;
    int J = 0;
    uint64_t seed = 0;
    int K = 0;
    bool park = false;  // stop after the initial build (sketch API)
    int pause_k = -1;   // stop before pick number pause_k (>= 0), parity hook
    Arena arena;
    uint8_t* M = nullptr;
    uint32_t* X = nullptr;
    uint32_t* Ju = nullptr;
    unsigned long long* Hu = nullptr;
    uint8_t* is_seed = nullptr;
    int32_t* best = nullptr;
    SweepDev sw{};
    CascadeDev c{};
    ArgmaxScratch am{};
    int32_t* seeds = nullptr;
    uint32_t* pickJ = nullptr;
    unsigned long long* pickH = nullptr;
    PropCounters* pc = nullptr;
    uint32_t* vstamp = nullptr;    // instrumented runs: per-row launch stamps
    uint32_t prop_launch_id = 0;   // instrumented runs: id of the last propagation launch
    // host state
    Stage stage = Stage::Fill;
    bool fresh = true;      // the next fill is the sketch's first: every register uncovered
    bool need_est = false;  // the next pick must recompute the estimate terms (after a build)
    int sweep = 0;
    int level = 1;
    uint32_t lv_pending = ~0u;    // level whose flags the next step must compact first (~0u: none)
    bool small_front = false;     // the last sweep (level) seen left a frontier small enough for a tail kernel
    int tail_kind = 0;            // this step: 1 tail sweeps, 2 tail levels, 0 none
    int nparts = 0;               // partials of the last argmax (the lazy argmax's partition)
    bool tails_ok = false;        // tail kernels may serve this query (engine tail mode and graph degrees)
    int32_t* chg_list2 = nullptr; // second in-task list of the tail sweeps
    int k = 0;
    uint32_t cascade_id = 0;
    uint64_t T_old = 0;
    std::vector<uint64_t> T;
    im_stats st{};
    double t_build0 = 0, t_sel0 = 0;
    int cap_K = 0;
};

class Engine {
public:
    Engine(hipStream_t st, int capacity, size_t budget) : st_(st), cap_(capacity), budget_(budget) {}
    ~Engine()
    {
        (void)hipStreamSynchronize(st_);  // no kernel may still use the buffers below
        drop_graph();
        if (gstream_) {
            (void)hipStreamSynchronize(gstream_);
            (void)hipStreamDestroy(gstream_);
        }
        for (Query* q : slots_)
            if (q) release(q);
        bufs_.release();
        if (status_host_) (void)hipHostFree(status_host_);
        if (args_host_) (void)hipHostFree(args_host_);
        for (auto& e : ev_)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : ph_)
            if (e) (void)hipEventDestroy(e);
    }

    im_status init()
    {
        if (cap_ < 1) return set_error(IM_EINVAL, "engine capacity must be >= 1");
        slots_.assign(cap_, nullptr);
        IMX_HIP(bufs_.alloc(&status_dev_, (size_t)cap_));
        IMX_HIP(hipMemsetAsync(status_dev_, 0, sizeof(SlotStatus) * cap_, st_));
        IMX_HIP(hipHostMalloc(reinterpret_cast<void**>(&status_host_), sizeof(SlotStatus) * cap_, 0));
        // argument records of one tick: at most kMaxRounds x (prep, propagate,
        // mark) or kMaxRounds x (level, compaction) plus a few per query, and
        // one 256-byte alignment per launch
        // Per query and step at most: per round prep, two propagation
        // records (graph mode with different kernels for the first and later
        // sweeps), mark, level and compaction; plus fill, estimate, argmax,
        // seed, tail prep, tail sweeps, pending compaction, tail levels and
        // finalize.  Every launch's array starts on 256 bytes.
        static_assert(sizeof(PrepArgs) + 2 * sizeof(PropArgs) + sizeof(MarkArgs) + sizeof(LevelArgs) +
                              sizeof(LevelCompactArgs) <= 6 * 384,
                      "round records");
        static_assert(sizeof(FillArgs) + sizeof(EstArgs) + sizeof(ArgmaxArgs) + sizeof(SeedArgs) + sizeof(PrepArgs) +
                              sizeof(TailSweepArgs) + sizeof(LevelCompactArgs) + sizeof(TailLevelArgs) +
                              sizeof(FinArgs) <= 9 * 384,
                      "step records");
        const size_t chunks = ((size_t)cap_ + kMaxBatch - 1) / kMaxBatch;
        args_cap_ = (size_t)cap_ * (kMaxRounds * 6 + 9) * 384 + chunks * (kMaxRounds * 6 + 9) * 256;
        IMX_HIP(bufs_.alloc(&args_dev_, args_cap_));
        IMX_HIP(hipHostMalloc(reinterpret_cast<void**>(&args_host_), args_cap_, 0));
        // timing-only events: no system-scope fence at record (a fenced record
        // costs a cache write-back and invalidation between kernels)
        for (auto& e : ev_) IMX_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        for (auto& e : ph_) IMX_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        // Environment overrides of the default tuning (validated like im_engine_set_tuning).
        im_tuning t = tune_;
        if (const char* v = std::getenv("IMX_GROUP_FIRST")) t.group_first = std::atoi(v);
        if (const char* v = std::getenv("IMX_GROUP")) t.group_rest = std::atoi(v);
        if (const char* v = std::getenv("IMX_ROUNDS")) t.rounds_per_step = std::atoi(v);
        if (const char* v = std::getenv("IMX_DENSE_DIV")) t.dense_div = std::atoi(v);
        if (const char* v = std::getenv("IMX_GRAPHS")) t.use_graphs = std::atoi(v);
        if (const char* v = std::getenv("IMX_TAIL")) t.tails = std::atoi(v);
        if (set_tuning(t) != IM_OK) return IM_EINVAL;
        // Cap on the workgroups of a propagation launch (schedule tests: few
        // workgroups make every one of them take many packs).
        // Tail kernels for small frontiers (on unless IMX_TAIL=0; limits by
        // environment for experiments).
        if (const char* v = std::getenv("IMX_TAIL_ROWS")) tail_rows_ = std::max(0, std::atoi(v));
        if (const char* v = std::getenv("IMX_TAIL_TASKS")) tail_tasks_ = std::max(1, std::atoi(v));
        if (const char* v = std::getenv("IMX_TAIL_ROUNDS")) tail_rounds_ = std::max(1, std::atoi(v));
        // Device-side workgroup splits for direct launches of several queries
        // (graph mode always uses them); IMX_DYN_SPLIT=0 keeps host splits.
        if (const char* v = std::getenv("IMX_DYN_SPLIT")) dyn_split_ = std::atoi(v) != 0;
        if (const char* v = std::getenv("IMX_PROP_GRID")) {
            prop_grid_cap_ = std::atoi(v);
            if (prop_grid_cap_ < 1) return set_error(IM_EINVAL, "IMX_PROP_GRID must be >= 1");
        }
        IMX_HIP(hipStreamSynchronize(st_));
        return IM_OK;
    }

    size_t used() const { return used_; }
    size_t budget() const { return budget_; }
    int active() const
    {
        int a = 0;
        for (Query* q : slots_)
            if (q && q->stage != Stage::Done && q->stage != Stage::Built && q->stage != Stage::Paused &&
                q->stage != Stage::Failed)
                ++a;
        return a;
    }

    // Device bytes one query would hold.
    static size_t footprint(const im_graph* g, int J, int K)
    {
        const size_t n = (size_t)g->n, nt = (size_t)std::max<int64_t>(g->ntasks, 1);
        const size_t nit = (size_t)std::max<int64_t>(g->n_in_tasks, 1), bmw = (n + 31) / 32;
        return n * (size_t)J + n * (4 + 8 + 1 + 4 * 2) + (size_t)flag_bytes((int64_t)n) * 2 +
               (size_t)blk_bytes((int64_t)n) * 2 + bmw * 8 + nt * 16 +
               nit * 8 + ((size_t)J + kTableWords) * 4 +
               (size_t)kArgmaxBlocks * 16 + (size_t)std::max(K, 1) * 16 + 4096;
    }

    im_status submit(const im_graph* g, int J, uint64_t seed, int K, bool park, Query** out)
    {
        *out = nullptr;
        if (!g) return set_error(IM_EINVAL, "graph is NULL");
        if (J < 64 || J > kMaxJ || J % 64 != 0) return set_error(IM_EINVAL, "J must be a multiple of 64 in [64, 4096]");
        if (!park && (K < 1 || K > g->n)) return set_error(IM_EINVAL, "K must be in [1, n]");
        int slot = -1;
        for (int i = 0; i < cap_; ++i)
            if (!slots_[i]) {
                slot = i;
                break;
            }
        if (slot < 0) return set_error(IM_ENOMEM, "engine has no free query slot");
        const size_t need = footprint(g, J, park ? 1 : K);
        if (used_ + need > budget_) return set_error(IM_ENOMEM, "query does not fit in the engine's memory budget");
        size_t free_b = 0, total_b = 0;
        IMX_HIP(hipMemGetInfo(&free_b, &total_b));
        if (need + (64u << 20) > free_b) return set_error(IM_ENOMEM, "query does not fit in device memory");

        auto q = std::make_unique<Query>();
        q->id = next_id_++;
        q->slot = slot;
        q->g = g;
        q->J = J;
        q->seed = seed;
        q->K = K;
        q->park = park;
        const int64_t n = g->n;
        const size_t nJ = (size_t)n * (size_t)J, bmw = (size_t)((n + 31) / 32);
        const size_t nt = (size_t)std::max<int64_t>(g->ntasks, 1), nit = (size_t)std::max<int64_t>(g->n_in_tasks, 1);
        Arena& A = q->arena;
        if (A.alloc(&q->M, nJ) || A.alloc(&q->X, (size_t)J + kTableWords) || A.alloc(&q->Ju, n) || A.alloc(&q->Hu, n) ||
            A.alloc(&q->sw.chg[0], bmw) || A.alloc(&q->sw.chg[1], bmw) || A.alloc(&q->sw.act8, flag_bytes(n)) ||
            A.alloc(&q->sw.act_tasks[0], nt) || A.alloc(&q->sw.act_tasks[1], nt) || A.alloc(&q->sw.chg_list, nit) ||
            A.alloc(&q->is_seed, n) || A.alloc(&q->best, 1) || A.alloc(&q->c.q[0], nt) || A.alloc(&q->c.q[1], nt) ||
            A.alloc(&q->c.lv8, flag_bytes(n)) || A.alloc(&q->c.touched, n) || A.alloc(&q->c.touch_stamp, n) ||
            A.alloc(&q->am.pJ, kArgmaxBlocks) || A.alloc(&q->am.pH, kArgmaxBlocks) || A.alloc(&q->am.pid, kArgmaxBlocks) ||
            A.alloc(&q->am.dirty, kArgmaxBlocks) ||
            A.alloc(&q->chg_list2, nit) || A.alloc(&q->sw.act_blk, blk_bytes(n)) || A.alloc(&q->c.lv_blk, blk_bytes(n))) {
            A.release();
            return set_error(IM_ENOMEM, "device allocation failed");
        }
        if (!park && alloc_results(q.get(), K) != IM_OK) {
            A.release();
            return IM_ENOMEM;
        }
        if (profiling_level() >= 2 && (A.alloc(&q->pc, 1) || A.alloc(&q->vstamp, n))) {
            A.release();
            return set_error(IM_ENOMEM, "device allocation failed");
        }
        SlotStatus* S = status_dev_ + slot;
        q->sw.rows_changed = S->rows_changed;
        q->sw.act_count = S->act_count;
        q->sw.chg_count = S->chg_count;
        q->sw.dense = S->dense;
        q->sw.conv = &S->conv;
        q->c.level_end = &S->level_end;
        q->c.qsize = S->qsize;
        q->c.T = &S->T;
        q->c.ntouched = &S->ntouched;

        hipError_t e = hipMemsetAsync(S, 0, sizeof(SlotStatus), st_);
        if (e == hipSuccess) e = hipMemsetAsync(q->is_seed, 0, n, st_);
        if (e == hipSuccess) e = hipMemsetAsync(q->am.dirty, 1, kArgmaxBlocks, st_);
        if (e == hipSuccess) e = hipMemsetAsync(q->sw.act8, 0, flag_bytes(n), st_);
        if (e == hipSuccess) e = hipMemsetAsync(q->c.lv8, 0, flag_bytes(n), st_);
        if (e == hipSuccess) e = hipMemsetAsync(q->sw.act_blk, 0, blk_bytes(n), st_);
        if (e == hipSuccess) e = hipMemsetAsync(q->c.lv_blk, 0, blk_bytes(n), st_);
        if (e == hipSuccess) e = hipMemsetAsync(q->c.touch_stamp, 0, sizeof(uint32_t) * n, st_);
        if (e == hipSuccess && q->pc) e = hipMemsetAsync(q->pc, 0, sizeof(PropCounters), st_);
        if (e == hipSuccess && q->vstamp) e = hipMemsetAsync(q->vstamp, 0, sizeof(uint32_t) * n, st_);
        if (e == hipSuccess) e = launch_sim_values(seed, J, q->X, st_);
        if (e != hipSuccess) {
            A.release();
            return set_error(IM_EDEVICE, std::string("query init: ") + hipGetErrorString(e));
        }
        q->stage = Stage::Fill;
        q->fresh = true;
        q->tails_ok = tune_.tails == 1 ||
                      (tune_.tails == 2 && std::max(g->max_out_deg, g->max_in_deg) <= kTailAutoDegree);
        q->t_build0 = now_ms();
        used_ += A.bytes;
        slots_[slot] = q.get();
        *out = q.release();
        return IM_OK;
    }

    im_status alloc_results(Query* q, int K)
    {
        if (q->arena.alloc(&q->seeds, K) || q->arena.alloc(&q->pickJ, K) || q->arena.alloc(&q->pickH, K))
            return set_error(IM_ENOMEM, "device allocation failed");
        q->T.assign(K, 0);
        q->cap_K = K;
        return IM_OK;
    }

    // A parked (built) query starts selecting K seeds, or a paused one goes on;
    // it stops again before pick `pause_k` (-1: runs to the end).
    im_status resume(Query* q, int K, int pause_k)
    {
        if (q->stage == Stage::Paused) {
            if (K != q->K) return set_error(IM_EINVAL, "K differs from the K of the paused selection");
            if (pause_k >= 0 && (pause_k < q->k || pause_k >= K))
                return set_error(IM_EINVAL, "pause pick must lie in [picks made, K)");
            q->pause_k = pause_k;
            enter_pick(q);
            return IM_OK;
        }
        if (q->stage != Stage::Built) return set_error(IM_ESTATE, "seeds were already selected on this sketch");
        if (K < 1 || K > q->g->n) return set_error(IM_EINVAL, "K must be in [1, n]");
        if (pause_k >= K) return set_error(IM_EINVAL, "pause pick must lie in [0, K)");
        const size_t before = q->arena.bytes;
        if (alloc_results(q, K) != IM_OK) return IM_ENOMEM;
        used_ += q->arena.bytes - before;
        q->K = K;
        q->park = false;
        q->pause_k = pause_k;
        q->t_sel0 = now_ms();
        enter_pick(q);
        return IM_OK;
    }

    // Next stage of a query whose next step is a pick: the pick itself, or a
    // pause before it (estimate terms first when a build just finished).
    static void enter_pick(Query* q)
    {
        if (q->pause_k >= 0 && q->k >= q->pause_k)
            q->stage = q->need_est ? Stage::Estimate : Stage::Paused;
        else
            q->stage = Stage::Pick;
    }

    // Seeds picked so far and T after each of their cascades.
    im_status partial_results(Query* q, int32_t* seeds, uint64_t* T)
    {
        if (q->k > 0 && seeds) {
            IMX_HIP(hipMemcpyAsync(seeds, q->seeds, sizeof(int32_t) * q->k, hipMemcpyDeviceToHost, st_));
            IMX_HIP(hipStreamSynchronize(st_));
        }
        if (T)
            for (int k = 0; k < q->k; ++k) T[k] = q->T[k];
        return IM_OK;
    }

    void release(Query* q)
    {
        if (q->slot >= 0 && q->slot < cap_ && slots_[q->slot] == q) slots_[q->slot] = nullptr;
        used_ -= std::min(used_, q->arena.bytes);
        q->arena.release();
    }

    void destroy(Query* q)
    {
        (void)hipStreamSynchronize(st_);
        release(q);
        delete q;
    }

    im_status step();

    // Step until no query is in a running stage.
    im_status run()
    {
        while (active() > 0)
            if (im_status e = step()) return e;
        return IM_OK;
    }

    im_status results(Query* q, int32_t* seeds, double* spread, double* est, uint64_t* T, im_stats* stats)
    {
        if (q->stage != Stage::Done) return set_error(IM_ESTATE, "query has not finished");
        const int K = q->K;
        std::vector<uint32_t> hJ(K);
        std::vector<unsigned long long> hH(K);
        std::vector<int32_t> hs(K);
        IMX_HIP(hipMemcpyAsync(hs.data(), q->seeds, sizeof(int32_t) * K, hipMemcpyDeviceToHost, st_));
        IMX_HIP(hipMemcpyAsync(hJ.data(), q->pickJ, sizeof(uint32_t) * K, hipMemcpyDeviceToHost, st_));
        IMX_HIP(hipMemcpyAsync(hH.data(), q->pickH, sizeof(unsigned long long) * K, hipMemcpyDeviceToHost, st_));
        IMX_HIP(hipStreamSynchronize(st_));
        for (int k = 0; k < K; ++k)
            if (hs[k] < 0) return set_error(IM_EDEVICE, "argmax found no candidate");
        if (seeds) std::memcpy(seeds, hs.data(), sizeof(int32_t) * K);
        if (est)
            for (int k = 0; k < K; ++k) est[k] = estimate_value(q->J, hJ[k], hH[k]);
        if (T)
            for (int k = 0; k < K; ++k) T[k] = q->T[k];
        if (spread) *spread = (double)q->T[K - 1] / (double)q->J;
        if (stats) *stats = q->st;
        return IM_OK;
    }

    hipStream_t stream() const { return st_; }

    im_status set_tuning(const im_tuning& t)
    {
        auto ok_gs = [](int v) { return v == 0 || v == 16 || v == 32 || v == 64; };
        if (!ok_gs(t.group_first) || !ok_gs(t.group_rest) || t.rounds_per_step < 1 ||
            t.rounds_per_step > kMaxRounds || t.dense_div < 1 || (t.use_graphs != 0 && t.use_graphs != 1) ||
            t.grid_cap < 0 || t.tails < 0 || t.tails > 2)
            return set_error(IM_EINVAL, "tuning out of range");
        tune_ = t;
        return IM_OK;
    }
    const im_tuning& tuning() const { return tune_; }
    void counters(int64_t* steps, int64_t* built, int64_t* replays) const
    {
        if (steps) *steps = steps_;
        if (built) *built = graphs_built_;
        if (replays) *replays = graph_replays_;
    }

private:
    // Argument records of one tick are packed into a pinned host buffer and
    // copied to the device once, before the tick's launches.
    template <class A>
    const A* stage_args(const std::vector<A>& v)
    {
        const size_t off = (args_off_ + 255) & ~size_t(255);
        const size_t nb = sizeof(A) * v.size();
        if (off + nb > args_cap_) return nullptr;
        std::memcpy(args_host_ + off, v.data(), nb);
        args_off_ = off + nb;
        return reinterpret_cast<const A*>(args_dev_ + off);
    }

    // Workgroup prefix for up to kMaxBatch queries, given per-query demands
    // and a cap on the launch's total (scaled down proportionally, >= 1 each).
    int64_t prop_cap(int64_t full) const { return prop_grid_cap_ > 0 ? std::min<int64_t>(full, prop_grid_cap_) : full; }

    static Batch make_batch(const std::vector<int64_t>& want, int64_t cap)
    {
        Batch B{};
        B.nq = (int)want.size();
        int64_t tot = 0;
        for (int64_t w : want) tot += std::max<int64_t>(w, 1);
        B.wg0[0] = 0;
        for (int i = 0; i < B.nq; ++i) {
            int64_t w = std::max<int64_t>(want[i], 1);
            if (cap > 0 && tot > cap) w = std::max<int64_t>(1, w * cap / tot);
            B.wg0[i + 1] = B.wg0[i] + (int)w;
        }
        return B;
    }

    template <class A>
    struct Launch {
        std::vector<A> args;
        std::vector<int64_t> want;
        const A* dev = nullptr;
        Batch B{};
        int maxJ = 0;
    };

    hipStream_t st_;
    int cap_;
    size_t budget_;
    int64_t prop_grid_cap_ = 0;  // IMX_PROP_GRID (0: none)
    bool dyn_split_ = true;      // IMX_DYN_SPLIT
    // Tail kernels: a query whose last sweep changed at most tail_rows_ rows
    // (or whose next level has at most tail_tasks_ tasks, or a new cascade)
    // runs up to tail_rounds_ sweeps (levels) in one single-workgroup launch;
    // the kernels hand back frontiers beyond tail_tasks_ tasks.
    // Tail mode 2 (default) serves graphs of bounded degree only: with hubs
    // (power-law graphs) a few changed rows have thousands of in-arcs, so
    // small frontiers rarely stay small for a single workgroup.
    static constexpr int64_t kTailAutoDegree = 64;
    int tail_rows_ = 64, tail_tasks_ = 64, tail_rounds_ = 256;
    size_t used_ = 0;
    int64_t next_id_ = 1;
    std::vector<Query*> slots_;
    Arena bufs_;  // the engine's own device buffers (status records, argument records)
    SlotStatus* status_dev_ = nullptr;
    SlotStatus* status_host_ = nullptr;
    uint8_t* args_dev_ = nullptr;
    uint8_t* args_host_ = nullptr;
    size_t args_cap_ = 0, args_off_ = 0;
    hipEvent_t ev_[2 * kMaxRounds] = {};
    hipEvent_t ph_[4] = {};  // sweep phase start/end, cascade phase start/end
    // graph mode: the instantiated graph of the last captured tick structure
    // graph mode: instantiated graphs of recent step structures (least
    // recently used dropped first)
    struct CachedGraph {
        std::vector<int64_t> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        int64_t last_use = 0;
    };
    static constexpr size_t kGraphCache = 8;
    std::vector<CachedGraph> graphs_;
    hipStream_t gstream_ = nullptr;  // private stream for graphs when the engine's stream is the null stream
    int64_t graphs_built_ = 0, graph_replays_ = 0, steps_ = 0;
    void drop_graph()
    {
        for (CachedGraph& c : graphs_) {
            if (c.exec) (void)hipGraphExecDestroy(c.exec);
            if (c.graph) (void)hipGraphDestroy(c.graph);
        }
        graphs_.clear();
    }
    im_tuning tune_{0, 0, 8, 16, 0, 0, 2};
};

im_status Engine::step()
{
    std::vector<Query*> act;
    for (Query* q : slots_)
        if (q && (q->stage == Stage::Fill || q->stage == Stage::Sweeps || q->stage == Stage::Estimate ||
                  q->stage == Stage::Pick || q->stage == Stage::Levels))
            act.push_back(q);
    if (act.empty()) return IM_OK;
    ++steps_;
    const int cus = device_cu_count();
    const int nr = tune_.rounds_per_step;
    const int gs_first_ = tune_.group_first, gs_rest_ = tune_.group_rest;
    args_off_ = 0;

    const bool stats = profiling_level() >= 2;
    // Small frontiers go to the tail kernels (not in instrumented runs, whose
    // counters cover the full-grid propagation kernel only).
    const bool tails = tune_.tails != 0 && !stats;
    std::vector<Query*> fill_q, sweep_q, est_q, pick_q, level_q, tailsw_q, taillv_q, cmp_q;
    for (Query* q : act) q->tail_kind = 0;
    for (Query* q : act) {
        switch (q->stage) {
        case Stage::Fill: fill_q.push_back(q); sweep_q.push_back(q); break;
        case Stage::Sweeps: (tails && q->tails_ok && q->small_front ? tailsw_q : sweep_q).push_back(q); break;
        case Stage::Estimate: est_q.push_back(q); break;
        case Stage::Pick:
            pick_q.push_back(q);
            (tails && q->tails_ok ? taillv_q : level_q).push_back(q);
            break;
        case Stage::Levels:
            if (q->lv_pending != ~0u) {
                cmp_q.push_back(q);
                level_q.push_back(q);
            } else {
                (tails && q->tails_ok && q->small_front ? taillv_q : level_q).push_back(q);
            }
            break;
        default: break;
        }
    }
    for (Query* q : pick_q) {
        ++q->cascade_id;
        q->level = 1;
    }

    // ---- build all launches (argument records) of this tick.  In graph mode
    // every launch list holds every running query, with the records of the
    // queries outside that launch's stage inactive: the launch sequence of a
    // step then depends only on the admitted queries, and its captured graph
    // replays until one finishes or another is admitted.
    const bool graph_mode = tune_.use_graphs != 0 && !stats;
    using Member = std::pair<Query*, bool>;
    auto members = [&](const std::vector<Query*>& v) {
        std::vector<Member> out;
        if (!graph_mode) {
            for (Query* q : v) out.push_back({q, true});
        } else {
            for (Query* q : act) out.push_back({q, std::find(v.begin(), v.end(), q) != v.end()});
        }
        return out;
    };
    // chunks of at most kMaxBatch records per launch
    auto mchunks = [](const std::vector<Member>& v) {
        std::vector<std::vector<Member>> out;
        for (size_t i = 0; i < v.size(); i += kMaxBatch)
            out.emplace_back(v.begin() + i, v.begin() + std::min(v.size(), i + kMaxBatch));
        return out;
    };
    auto with = [](auto rec, bool active) {
        rec.active = active ? 1 : 0;
        return rec;
    };
    for (Query* q : tailsw_q) q->tail_kind = 1;
    for (Query* q : taillv_q) q->tail_kind = 2;

    std::vector<Launch<FillArgs>> L_fill;
    for (auto& ch : mchunks(members(fill_q))) {
        Launch<FillArgs> L;
        for (auto [q, on] : ch) {
            L.args.push_back(with(FillArgs{q->M, q->g->n, q->J, q->fresh ? 1 : 0, q->seed}, on));
            const int64_t rows_per_wg = 256 / row_lanes(q->J);
            L.want.push_back(std::min<int64_t>(cus * 16, (q->g->n + rows_per_wg - 1) / rows_per_wg));
        }
        L_fill.push_back(std::move(L));
    }
    struct SweepRound {
        std::vector<Launch<PrepArgs>> prep;
        std::vector<Launch<PropArgs>> prop_first, prop_rest;
        std::vector<Launch<MarkArgs>> mark;
    };
    const std::vector<Member> sweep_m = members(sweep_q);
    std::vector<SweepRound> rounds(sweep_m.empty() ? 0 : nr);
    int full_first = 0, full_rest = 0;
    if (!sweep_m.empty()) {
        int maxJ = 0;
        for (auto [q, on] : sweep_m) maxJ = std::max(maxJ, q->J);
        IMX_HIP(propagate_full_grid(maxJ, gs_first_, stats, &full_first));
        IMX_HIP(propagate_full_grid(maxJ, gs_rest_, stats, &full_rest));
    }
    // graph mode with one kernel choice for all sweeps: a single propagation list
    const bool one_prop_list = graph_mode && gs_first_ == gs_rest_;
    for (int b = 0; b < (int)rounds.size(); ++b) {
        for (auto& ch : mchunks(sweep_m)) {
            Launch<PrepArgs> P;
            Launch<PropArgs> F, R;
            Launch<MarkArgs> K;
            for (auto [q, on] : ch) {
                const int s = q->sweep + b;
                const GraphDev gd = q->g->dev();
                const int64_t nwords = (q->g->n + 31) / 32;
                P.args.push_back(with(PrepArgs{q->sw, q->g->task_start, q->g->n, nwords, s}, on));
                P.want.push_back(std::min<int64_t>(cus * 4, (q->g->n + 16 * kWG - 1) / (16 * kWG)));
                PropArgs pa{gd,
                            q->X,
                            q->J,
                            q->M,
                            s == 0 ? nullptr : q->sw.act_tasks[s & 1],
                            &q->sw.act_count[s & 3],
                            q->sw.chg[s & 1],
                            q->sw.chg[(s + 1) & 1],
                            q->sw.chg_list,
                            &q->sw.chg_count[s & 3],
                            &q->sw.dense[s & 3],
                            q->sw.conv,
                            &q->sw.rows_changed[s & 3],
                            q->pc,
                            q->vstamp,
                            on ? ++q->prop_launch_id : q->prop_launch_id};
                auto add_prop = [&](Launch<PropArgs>& T, int gsel, bool act_here) {
                    const int lanes = propagate_group_size(q->J, gsel), thr = propagate_wg_threads(gsel);
                    T.args.push_back(with(pa, act_here));
                    T.want.push_back((q->g->ntasks * lanes + thr - 1) / thr);
                    T.maxJ = std::max(T.maxJ, q->J);
                };
                if (one_prop_list) {
                    add_prop(R, gs_rest_, on);
                } else if (graph_mode) {
                    add_prop(F, gs_first_, on && s == 0);
                    add_prop(R, gs_rest_, on && s != 0);
                } else {
                    add_prop(s == 0 ? F : R, s == 0 ? gs_first_ : gs_rest_, on);
                }
                K.args.push_back(with(MarkArgs{gd, q->sw, s, tune_.dense_div}, on));
                K.want.push_back(std::min<int64_t>(cus * 4, (q->g->n_in_tasks + kWaves - 1) / kWaves));
            }
            rounds[b].prep.push_back(std::move(P));
            if (!F.args.empty()) rounds[b].prop_first.push_back(std::move(F));
            if (!R.args.empty()) rounds[b].prop_rest.push_back(std::move(R));
            rounds[b].mark.push_back(std::move(K));
        }
    }
    std::vector<Launch<EstArgs>> L_est;
    std::vector<Query*> est_all = est_q;
    for (Query* q : pick_q)
        if (q->need_est) est_all.push_back(q);  // estimate terms after every build
    for (auto& ch : mchunks(members(est_all))) {
        Launch<EstArgs> L;
        for (auto [q, on] : ch) {
            L.args.push_back(with(EstArgs{q->M, q->g->n, q->J, q->Ju, q->Hu, q->am.dirty}, on));
            const int64_t rows_per_wg = kWG / row_lanes(q->J) * kRowBatch;
            L.want.push_back(std::min<int64_t>(cus * 16, (q->g->n + rows_per_wg - 1) / rows_per_wg));
        }
        L_est.push_back(std::move(L));
    }
    std::vector<Launch<ArgmaxArgs>> L_am;
    std::vector<Launch<SeedArgs>> L_seed;
    for (auto& ch : mchunks(members(pick_q))) {
        Launch<ArgmaxArgs> L;
        Launch<SeedArgs> S;
        for (auto [q, on] : ch) {
            // graph mode: few partial workgroups per query (every query's are launched every step)
            const int nparts =
                (int)std::min<int64_t>(graph_mode ? kGraphArgmaxBlocks : kArgmaxBlocks, (q->g->n + 255) / 256);
            // a change of the partition (graph mode switched) makes every partial stale
            ArgmaxScratch am = q->am;
            if (on && std::max(nparts, 1) != q->nparts) {
                am.dirty = nullptr;
                q->nparts = std::max(nparts, 1);
            }
            L.args.push_back(with(ArgmaxArgs{q->Ju, q->Hu, q->is_seed, q->g->n, am, q->best, std::max(nparts, 1)}, on));
            L.want.push_back(std::max(nparts, 1));
            S.args.push_back(with(SeedArgs{q->g->dev(), q->best, q->k, q->M, q->J, q->is_seed, q->seeds, q->pickJ,
                                           q->pickH, q->Ju, q->Hu, q->c, q->cascade_id},
                                  on));
            S.want.push_back(1);
        }
        L_am.push_back(std::move(L));
        L_seed.push_back(std::move(S));
    }
    const std::vector<Member> level_m = members(level_q);
    std::vector<std::vector<Launch<LevelArgs>>> L_lvl(level_m.empty() ? 0 : nr);
    std::vector<std::vector<Launch<LevelCompactArgs>>> L_cmp(level_m.empty() ? 0 : nr);
    int full_level = 0;
    if (!level_m.empty()) {
        int maxJ = 0;
        for (auto [q, on] : level_m) maxJ = std::max(maxJ, q->J);
        IMX_HIP(cascade_level_full_grid(maxJ, &full_level));
    }
    for (int b = 0; b < (int)L_lvl.size(); ++b)
        for (auto& ch : mchunks(level_m)) {
            Launch<LevelArgs> L;
            Launch<LevelCompactArgs> C;
            for (auto [q, on] : ch) {
                const int t = q->level + b;
                L.args.push_back(with(LevelArgs{q->g->dev(), q->X, q->J, q->M, q->c, t}, on));
                L.want.push_back((q->g->ntasks + kWaves - 1) / kWaves);
                L.maxJ = std::max(L.maxJ, q->J);
                C.args.push_back(with(LevelCompactArgs{q->g->task_start, q->g->n, q->c, t, q->cascade_id}, on));
                C.want.push_back(std::min<int64_t>(cus * 4, (q->g->n + 16 * kWG - 1) / (16 * kWG)));
            }
            L_lvl[b].push_back(std::move(L));
            L_cmp[b].push_back(std::move(C));
        }
    // finalize (it runs only once a cascade has ended), for the queries in
    // full-grid levels and in tail levels
    std::vector<Query*> fin_q = level_q;
    fin_q.insert(fin_q.end(), taillv_q.begin(), taillv_q.end());
    std::vector<Launch<FinArgs>> L_fin;
    for (auto& ch : mchunks(members(fin_q))) {
        Launch<FinArgs> L;
        for (auto [q, on] : ch) {
            // no partition yet (no pick made): no lazy flags to keep
            L.args.push_back(
                with(FinArgs{q->M, q->J, q->Ju, q->Hu, q->c, q->nparts > 0 ? q->am.dirty : nullptr, q->nparts}, on));
            L.want.push_back(std::min<int64_t>(cus * 8, (q->g->n + 4 * kWaves - 1) / (4 * kWaves)));
        }
        L_fin.push_back(std::move(L));
    }

    // tail sweeps: the prep step of the first sweep, then the tail kernel
    std::vector<Launch<PrepArgs>> L_tprep;
    std::vector<Launch<TailSweepArgs>> L_tsw;
    for (auto& ch : mchunks(members(tailsw_q))) {
        Launch<PrepArgs> P;
        Launch<TailSweepArgs> T;
        for (auto [q, on] : ch) {
            const int s0 = q->sweep;
            const int64_t nwords = (q->g->n + 31) / 32;
            P.args.push_back(with(PrepArgs{q->sw, q->g->task_start, q->g->n, nwords, s0}, on));
            P.want.push_back(std::min<int64_t>(cus * 4, (q->g->n + 16 * kWG - 1) / (16 * kWG)));
            SlotStatus* S = status_dev_ + q->slot;
            T.args.push_back(with(TailSweepArgs{q->g->dev(), q->X, q->J, q->M, q->sw, q->chg_list2, &S->tail_next, s0,
                                                tail_rounds_, tune_.dense_div, (int64_t)kTailCap,
                                                (int64_t)tail_tasks_, &S->tail_reason},
                                  on));
            T.want.push_back(1);
            T.maxJ = std::max(T.maxJ, q->J);
        }
        L_tprep.push_back(std::move(P));
        L_tsw.push_back(std::move(T));
    }
    // pending compactions (a tail-levels launch flagged a level's heads)
    std::vector<Launch<LevelCompactArgs>> L_pcmp;
    for (auto& ch : mchunks(members(cmp_q))) {
        Launch<LevelCompactArgs> C;
        for (auto [q, on] : ch) {
            C.args.push_back(
                with(LevelCompactArgs{q->g->task_start, q->g->n, q->c, on ? (int)q->lv_pending : 0, q->cascade_id}, on));
            C.want.push_back(std::min<int64_t>(cus * 4, (q->g->n + 16 * kWG - 1) / (16 * kWG)));
            if (on) q->lv_pending = ~0u;
        }
        L_pcmp.push_back(std::move(C));
    }
    // tail levels: a new cascade (after its seed step) or a small frontier
    std::vector<Launch<TailLevelArgs>> L_tlv;
    for (auto& ch : mchunks(members(taillv_q))) {
        Launch<TailLevelArgs> T;
        for (auto [q, on] : ch) {
            SlotStatus* S = status_dev_ + q->slot;
            T.args.push_back(with(TailLevelArgs{q->g->dev(), q->X, q->J, q->M, q->c, &S->lv_next, &S->cmp_pending,
                                                q->level, tail_rounds_, (uint32_t)tail_tasks_, q->cascade_id,
                                                &S->tail_reason},
                                  on));
            T.want.push_back(1);
            T.maxJ = std::max(T.maxJ, q->J);
        }
        L_tlv.push_back(std::move(T));
    }

    // ---- stage argument records, one copy; the tick's launch structure
    // (kinds, grids, batch splits, record offsets) forms its graph key
    std::vector<int64_t> key;
    // Launches of several queries (and every launch in graph mode) split
    // their workgroups among the queries on the device, by each query's
    // current work (inactive queries get none): the host's split by graph
    // size ignores how much of a graph a sweep or level touches, and in graph
    // mode the fixed launch sequence would starve the active queries.  The
    // argmax (its partial count per query is fixed), the seed step and the
    // tail kernels (one workgroup per query) keep host splits.
    auto dynamic_kind = [](int kind) { return kind != 6 && kind != 7 && kind != 12 && kind != 14; };
    auto finish = [&](int kind, auto& L, int64_t cap) -> bool {
        L.dev = stage_args(L.args);
        if (tune_.grid_cap > 0 && kind != 6)  // the partial argmax keeps its per-query partial count
            cap = cap > 0 ? std::min<int64_t>(cap, tune_.grid_cap) : tune_.grid_cap;
        if ((graph_mode || (dyn_split_ && L.args.size() > 1)) && dynamic_kind(kind)) {
            L.B = Batch{};
            L.B.nq = (int)L.args.size();
            L.B.wg0[0] = -1;
            L.B.wg0[L.B.nq] = (int)std::max<int64_t>(cap > 0 ? cap : (int64_t)cus * 8, L.B.nq);
        } else {
            L.B = make_batch(L.want, cap);
        }
        key.push_back(kind);
        key.push_back(L.dev ? reinterpret_cast<const uint8_t*>(L.dev) - args_dev_ : -1);
        key.push_back(L.maxJ);
        key.push_back(L.B.nq);
        for (int i = 0; i <= L.B.nq; ++i) key.push_back(L.B.wg0[i]);
        return L.dev != nullptr;
    };
    // graph mode launches every query's workgroups for every kind: the grids of
    // the grid-stride kernels are capped in total (split by query size)
    const int64_t gcap = graph_mode ? (int64_t)cus * 8 : 0;
    bool ok = true;
    for (auto& L : L_fill) ok &= finish(0, L, gcap);
    for (auto& R : rounds) {
        for (auto& L : R.prep) ok &= finish(1, L, gcap);
        for (auto& L : R.prop_first) ok &= finish(2, L, prop_cap(full_first));
        for (auto& L : R.prop_rest) ok &= finish(3, L, prop_cap(full_rest));
        for (auto& L : R.mark) ok &= finish(4, L, (int64_t)cus * 4);
    }
    for (auto& L : L_est) ok &= finish(5, L, gcap);
    for (auto& L : L_am) ok &= finish(6, L, 0);
    for (auto& L : L_seed) ok &= finish(7, L, 0);
    for (auto& R : L_lvl)
        for (auto& L : R) ok &= finish(8, L, full_level);
    for (auto& R : L_cmp)
        for (auto& L : R) ok &= finish(9, L, gcap);
    for (auto& L : L_fin) ok &= finish(10, L, gcap);
    auto one_each = [](auto& L) {  // tail kernels: one workgroup per query
        for (int i = 0; i <= L.B.nq; ++i) L.B.wg0[i] = i;
    };
    for (auto& L : L_tprep) ok &= finish(11, L, gcap);
    for (auto& L : L_tsw) {
        ok &= finish(12, L, 0);
        one_each(L);
    }
    for (auto& L : L_pcmp) ok &= finish(13, L, gcap);
    for (auto& L : L_tlv) {
        ok &= finish(14, L, 0);
        one_each(L);
    }
    if (!ok) return set_error(IM_EINVAL, "too many queries for one tick's argument buffer");

    // ---- the tick's work, in dependency order: argument records in, kernels,
    // status records out.  `timed` adds the HIP events of the per-phase and
    // per-launch times (not recorded in graph mode).
    const bool sweeping = !rounds.empty() || !L_tsw.empty(), cascading = !L_lvl.empty() || !L_tlv.empty();
    int ne = 0;
    auto issue = [&](bool timed, hipStream_t sx) -> hipError_t {
        hipError_t e = hipMemcpyAsync(args_dev_, args_host_, args_off_, hipMemcpyHostToDevice, sx);
        auto ev = [&](hipEvent_t x) {
            if (timed && e == hipSuccess) e = hipEventRecord(x, sx);
        };
        if (sweeping) ev(ph_[0]);
        for (auto& L : L_fill)
            if (e == hipSuccess) e = launch_fill(L.dev, L.B, sx);
        for (auto& L : L_tprep)
            if (e == hipSuccess) e = launch_sweep_prep(L.dev, L.B, sx);
        for (auto& L : L_tsw)
            if (e == hipSuccess) e = launch_tail_sweeps(L.dev, L.B, L.maxJ, sx);
        for (auto& R : rounds) {
            for (auto& L : R.prep)
                if (e == hipSuccess) e = launch_sweep_prep(L.dev, L.B, sx);
            ev(ev_[2 * ne]);
            for (auto& L : R.prop_first)
                if (e == hipSuccess) e = launch_propagate(L.dev, L.B, L.maxJ, gs_first_, stats, sx);
            for (auto& L : R.prop_rest)
                if (e == hipSuccess) e = launch_propagate(L.dev, L.B, L.maxJ, gs_rest_, stats, sx);
            ev(ev_[2 * ne + 1]);
            ++ne;
            for (auto& L : R.mark)
                if (e == hipSuccess) e = launch_mark(L.dev, L.B, sx);
        }
        if (sweeping) ev(ph_[1]);
        for (auto& L : L_est)
            if (e == hipSuccess) e = launch_estimate(L.dev, L.B, sx);
        if (cascading) ev(ph_[2]);
        for (size_t i = 0; i < L_am.size(); ++i) {
            Batch fin{};
            fin.nq = L_am[i].B.nq;
            for (int j = 0; j <= fin.nq; ++j) fin.wg0[j] = j;
            if (e == hipSuccess) e = launch_argmax(L_am[i].dev, L_am[i].B, fin, sx);
            if (e == hipSuccess) e = launch_cascade_seed(L_seed[i].dev, L_seed[i].B, sx);
        }
        for (auto& L : L_tlv)
            if (e == hipSuccess) e = launch_tail_levels(L.dev, L.B, L.maxJ, sx);
        for (auto& L : L_pcmp)
            if (e == hipSuccess) e = launch_cascade_compact(L.dev, L.B, sx);
        for (size_t b = 0; b < L_lvl.size(); ++b) {
            for (auto& L : L_lvl[b])
                if (e == hipSuccess) e = launch_cascade_level(L.dev, L.B, L.maxJ, sx);
            for (auto& L : L_cmp[b])
                if (e == hipSuccess) e = launch_cascade_compact(L.dev, L.B, sx);
        }
        for (auto& L : L_fin)
            if (e == hipSuccess) e = launch_cascade_finalize(L.dev, L.B, sx);
        if (cascading) ev(ph_[3]);
        if (e == hipSuccess)
            e = hipMemcpyAsync(status_host_, status_dev_, sizeof(SlotStatus) * cap_, hipMemcpyDeviceToHost, sx);
        return e;
    };

    const bool timed = !graph_mode && profiling_level() >= 1;  // per-launch and per-phase events
    hipStream_t cs = st_;  // stream of this tick's work
    if (graph_mode) {
        key.push_back((int64_t)args_off_);
        key.push_back(gs_first_);
        key.push_back(gs_rest_);
        // the legacy null stream cannot be captured: use a private blocking
        // stream then (implicitly ordered with the null stream)
        if (!st_ && !gstream_) IMX_HIP(hipStreamCreate(&gstream_));
        cs = st_ ? st_ : gstream_;
        CachedGraph* hit = nullptr;
        for (CachedGraph& c : graphs_)
            if (c.key == key) hit = &c;
        if (!hit) {  // capture this structure once
            if (graphs_.size() >= kGraphCache) {  // drop the least recently used
                auto lru = std::min_element(graphs_.begin(), graphs_.end(),
                                            [](const CachedGraph& x, const CachedGraph& y) { return x.last_use < y.last_use; });
                if (lru->exec) (void)hipGraphExecDestroy(lru->exec);
                if (lru->graph) (void)hipGraphDestroy(lru->graph);
                graphs_.erase(lru);
            }
            IMX_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            const hipError_t e = issue(false, cs);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return set_error(IM_EDEVICE, std::string("graph capture: ") +
                                                 hipGetErrorString(e != hipSuccess ? e : e2));
            }
            CachedGraph c;
            c.key = key;
            c.graph = g;
            const hipError_t ei = hipGraphInstantiate(&c.exec, g, nullptr, nullptr, 0);
            if (ei != hipSuccess) {
                (void)hipGraphDestroy(g);
                return set_error(IM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
            }
            graphs_.push_back(c);
            hit = &graphs_.back();
            ++graphs_built_;
        }
        hit->last_use = steps_;
        IMX_HIP(hipGraphLaunch(hit->exec, cs));
        ++graph_replays_;
    } else {
        IMX_HIP(issue(timed, st_));
    }
    IMX_HIP(hipStreamSynchronize(cs));

    float sweep_phase_ms = 0.f, cascade_phase_ms = 0.f;
    if (timed && sweeping) (void)hipEventElapsedTime(&sweep_phase_ms, ph_[0], ph_[1]);
    if (timed && cascading) (void)hipEventElapsedTime(&cascade_phase_ms, ph_[2], ph_[3]);
    float prop_ms = 0.f;
    for (int i = 0; i < (timed ? ne : 0); ++i) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev_[2 * i], ev_[2 * i + 1]);
        prop_ms += ms;
    }

    // ---- advance every query's state machine
    for (Query* q : act) {
        const SlotStatus& S = status_host_[q->slot];
        switch (q->stage) {
        case Stage::Fill:
        case Stage::Sweeps: {
            q->st.propagate_ms += sweep_phase_ms;
            if (q->tail_kind == 1) {
                q->sweep = (int)S.tail_next;
            } else {
                q->st.prop_kernel_ms += prop_ms / (double)sweep_q.size();
                q->st.prop_launches += nr;
                q->sweep += nr;
            }
            if (S.conv != ~0u) {  // sweep S.conv (0-based) changed nothing: the build is complete
                const int sweeps = (int)S.conv + 1;
                q->st.total_sweeps += sweeps;
                if (q->fresh) {
                    q->st.build_sweeps = sweeps;
                    q->st.build_ms = now_ms() - q->t_build0;
                    q->t_sel0 = now_ms();
                }
                q->fresh = false;
                q->sweep = 0;
                q->need_est = true;
                if (q->park)
                    q->stage = Stage::Estimate;
                else
                    enter_pick(q);
            } else if (q->sweep > q->g->n + 2) {
                q->stage = Stage::Failed;
                return set_error(IM_EDEVICE, "propagation did not converge");
            } else {
                q->stage = Stage::Sweeps;
                q->small_front = (q->tail_kind == 1)
                                     ? S.tail_reason == kTailStopRounds
                                     : (S.dense[q->sweep & 3] == 0u &&
                                        S.rows_changed[(q->sweep - 1) & 3] <= (unsigned long long)tail_rows_);
            }
            break;
        }
        case Stage::Estimate:
            q->need_est = false;
            if (q->park) {
                q->stage = Stage::Built;
                q->st.build_ms = now_ms() - q->t_build0;
            } else {
                q->stage = Stage::Paused;  // estimate terms for a pause after a rebuild
            }
            break;
        case Stage::Pick:
        case Stage::Levels: {
            q->need_est = false;
            q->st.cascade_ms += cascade_phase_ms;
            if (q->tail_kind == 2) {
                q->level = (int)S.lv_next;
                q->lv_pending = S.cmp_pending;
            } else {
                q->level += nr;
            }
            if (S.level_end != ~0u) {  // the cascade ended and was finalized in this tick
                q->st.cascade_levels += S.level_end - 1u;
                const uint64_t T = S.T;
                q->T[q->k] = T;
                ++q->k;
                if (q->k >= q->K) {
                    q->stage = Stage::Done;
                    q->st.select_ms = now_ms() - q->t_sel0;
                } else if (100 * (T - q->T_old) > T) {
                    q->T_old = T;
                    ++q->st.rebuilds;
                    q->stage = Stage::Fill;
                    q->sweep = 0;
                    q->small_front = false;
                } else {
                    enter_pick(q);
                }
            } else if (q->level > q->g->n + 8) {
                q->stage = Stage::Failed;
                return set_error(IM_EDEVICE, "cascade did not terminate");
            } else {
                q->stage = Stage::Levels;
                q->small_front = (q->tail_kind == 2) ? S.tail_reason == kTailStopRounds
                                                     : S.qsize[q->level & 3] <= (uint32_t)tail_tasks_;
            }
            break;
        }
        default: break;
        }
    }
    return IM_OK;
}

}  // namespace imx

using imx::Engine;
using imx::Query;

// ---------------------------------------------------------------------------
// Sketches: one-query engines.

struct im_sketch {
    std::unique_ptr<Engine> eng;
    Query* q = nullptr;
    ~im_sketch()
    {
        if (q) eng->destroy(q);
    }
};

struct im_engine {
    std::unique_ptr<Engine> eng;
    std::vector<Query*> queries;
};

namespace {

im_status finish_prop_counters(Query* q)
{
    if (!q->pc) return IM_OK;
    imx::PropCounters c{};
    IMX_HIP(hipMemcpy(&c, q->pc, sizeof(c), hipMemcpyDeviceToHost));
    im_stats& s = q->st;
    s.prop_tasks = (int64_t)c.tasks;
    s.prop_rows_read = (int64_t)c.rows_read;
    s.prop_bytes_written = (int64_t)c.bytes_written;
    s.prop_arcs_scanned = (int64_t)c.arcs_scanned;
    s.prop_arcs_active = (int64_t)c.arcs_active;
    s.prop_sectors = (int64_t)c.sectors;
    s.prop_rows_visited = (int64_t)c.rows_visited;
    s.prop_rows_changed = (int64_t)c.rows_changed;
    // per sweep: (8 + J) per active row (row bounds, own registers), J per
    // changed row (stored), 8 + 64 per active arc and sector (head id,
    // threshold, the head's 64-byte sectors holding live registers)
    const double J = (double)q->J;
    s.prop_alg_bytes = (8.0 + J) * (double)c.rows_visited + J * (double)c.rows_changed + 8.0 * (double)c.arcs_active +
                       64.0 * (double)c.sectors;
    return IM_OK;
}

size_t device_free()
{
    size_t f = 0, t = 0;
    (void)hipMemGetInfo(&f, &t);
    return f;
}

}  // namespace

extern "C" {

im_status im_sketch_build(const im_graph* g, int32_t J, uint64_t seed, void* stream, im_sketch** out)
{
    if (!out) return imx::set_error(IM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return imx::set_error(IM_EINVAL, "graph is NULL");
    auto s = std::make_unique<im_sketch>();
    s->eng = std::make_unique<Engine>(static_cast<hipStream_t>(stream), 1, device_free());
    if (im_status e = s->eng->init()) return e;
    if (im_status e = s->eng->submit(g, J, seed, 0, true, &s->q)) return e;
    if (im_status e = s->eng->run()) return e;
    *out = s.release();
    return IM_OK;
}

im_status im_select_seeds(im_sketch* s, int32_t K, int32_t* seeds_host, double* spread_out, double* est_host,
                          uint64_t* T_host, im_stats* stats_out)
{
    if (!s) return imx::set_error(IM_EINVAL, "sketch is NULL");
    if (!seeds_host) return imx::set_error(IM_EINVAL, "seeds output is NULL");
    if (im_status e = s->eng->resume(s->q, K, -1)) return e;
    if (im_status e = s->eng->run()) return e;
    if (im_status e = finish_prop_counters(s->q)) return e;
    return s->eng->results(s->q, seeds_host, spread_out, est_host, T_host, stats_out);
}

im_status im_select_seeds_until(im_sketch* s, int32_t K, int32_t k_stop, int32_t* seeds_host, uint64_t* T_host)
{
    if (!s) return imx::set_error(IM_EINVAL, "sketch is NULL");
    if (k_stop < 0) return imx::set_error(IM_EINVAL, "k_stop must be >= 0");
    if (im_status e = s->eng->resume(s->q, K, k_stop)) return e;
    if (im_status e = s->eng->run()) return e;
    return s->eng->partial_results(s->q, seeds_host, T_host);
}

im_status im_sketch_registers(const im_sketch* s, uint8_t* regs_host)
{
    if (!s || !regs_host) return imx::set_error(IM_EINVAL, "NULL argument");
    IMX_HIP(hipMemcpyAsync(regs_host, s->q->M, (size_t)s->q->g->n * (size_t)s->q->J, hipMemcpyDeviceToHost,
                           s->eng->stream()));
    IMX_HIP(hipStreamSynchronize(s->eng->stream()));
    return IM_OK;
}

im_status im_sketch_register_rows(const im_sketch* s, const int32_t* rows_host, int32_t nrows, uint8_t* regs_host)
{
    if (!s || nrows < 0 || (nrows > 0 && (!rows_host || !regs_host))) return imx::set_error(IM_EINVAL, "NULL argument");
    for (int32_t i = 0; i < nrows; ++i)
        if (rows_host[i] < 0 || rows_host[i] >= s->q->g->n) return imx::set_error(IM_EINVAL, "row id out of range");
    const size_t J = (size_t)s->q->J;
    for (int32_t i = 0; i < nrows; ++i)
        IMX_HIP(hipMemcpyAsync(regs_host + (size_t)i * J, s->q->M + (size_t)rows_host[i] * J, J, hipMemcpyDeviceToHost,
                               s->eng->stream()));
    IMX_HIP(hipStreamSynchronize(s->eng->stream()));
    return IM_OK;
}

im_status im_sketch_estimates(const im_sketch* s, uint32_t* Ju_host, uint64_t* Hu_host)
{
    if (!s) return imx::set_error(IM_EINVAL, "sketch is NULL");
    const int64_t n = s->q->g->n;
    if (Ju_host)
        IMX_HIP(hipMemcpyAsync(Ju_host, s->q->Ju, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s->eng->stream()));
    if (Hu_host)
        IMX_HIP(hipMemcpyAsync(Hu_host, s->q->Hu, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s->eng->stream()));
    IMX_HIP(hipStreamSynchronize(s->eng->stream()));
    return IM_OK;
}

im_status im_sketch_stats(const im_sketch* s, im_stats* out)
{
    if (!s || !out) return imx::set_error(IM_EINVAL, "NULL argument");
    *out = s->q->st;
    return IM_OK;
}

im_status im_sketch_sim_values(const im_sketch* s, uint32_t* X_host)
{
    if (!s || !X_host) return imx::set_error(IM_EINVAL, "NULL argument");
    IMX_HIP(hipMemcpyAsync(X_host, s->q->X, sizeof(uint32_t) * s->q->J, hipMemcpyDeviceToHost, s->eng->stream()));
    IMX_HIP(hipStreamSynchronize(s->eng->stream()));
    return IM_OK;
}

void im_sketch_free(im_sketch* s) { delete s; }

// ---------------------------------------------------------------------------
// Engines (batched and continuously admitted queries).

im_status im_engine_create(int32_t max_queries, uint64_t hbm_budget_bytes, void* stream, im_engine** out)
{
    if (!out) return imx::set_error(IM_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_queries < 1 || max_queries > 4096) return imx::set_error(IM_EINVAL, "max_queries must be in [1, 4096]");
    auto e = std::make_unique<im_engine>();
    const size_t budget = hbm_budget_bytes ? (size_t)hbm_budget_bytes : device_free();
    e->eng = std::make_unique<Engine>(static_cast<hipStream_t>(stream), max_queries, budget);
    if (im_status st = e->eng->init()) return st;
    *out = e.release();
    return IM_OK;
}

im_status im_engine_submit(im_engine* e, const im_graph* g, int32_t J, uint64_t seed, int32_t K, int64_t* query_id)
{
    if (!e || !query_id) return imx::set_error(IM_EINVAL, "NULL argument");
    Query* q = nullptr;
    if (im_status st = e->eng->submit(g, J, seed, K, false, &q)) return st;
    e->queries.push_back(q);
    *query_id = q->id;
    return IM_OK;
}

im_status im_engine_step(im_engine* e, int32_t* n_running)
{
    if (!e) return imx::set_error(IM_EINVAL, "engine is NULL");
    if (im_status st = e->eng->step()) return st;
    if (n_running) *n_running = e->eng->active();
    return IM_OK;
}

im_status im_engine_poll(im_engine* e, int64_t* done_ids, int32_t capacity, int32_t* n_done)
{
    if (!e || !n_done || (capacity > 0 && !done_ids)) return imx::set_error(IM_EINVAL, "NULL argument");
    int32_t c = 0;
    for (Query* q : e->queries)
        if (q->stage == imx::Stage::Done) {
            if (c < capacity) done_ids[c] = q->id;
            ++c;
        }
    *n_done = c;
    return IM_OK;
}

im_status im_engine_result(im_engine* e, int64_t query_id, int32_t* seeds_host, double* spread_out,
                           double* est_host, uint64_t* T_host, im_stats* stats_out)
{
    if (!e || !seeds_host) return imx::set_error(IM_EINVAL, "NULL argument");
    for (size_t i = 0; i < e->queries.size(); ++i) {
        Query* q = e->queries[i];
        if (q->id != query_id) continue;
        if (im_status st = finish_prop_counters(q)) return st;
        if (im_status st = e->eng->results(q, seeds_host, spread_out, est_host, T_host, stats_out)) return st;
        e->eng->destroy(q);
        e->queries.erase(e->queries.begin() + (ptrdiff_t)i);
        return IM_OK;
    }
    return imx::set_error(IM_EINVAL, "unknown query id");
}

im_status im_engine_info(const im_engine* e, int32_t* n_queries, int32_t* n_running, uint64_t* bytes_used,
                         uint64_t* bytes_budget)
{
    if (!e) return imx::set_error(IM_EINVAL, "engine is NULL");
    if (n_queries) *n_queries = (int32_t)e->queries.size();
    if (n_running) *n_running = e->eng->active();
    if (bytes_used) *bytes_used = e->eng->used();
    if (bytes_budget) *bytes_budget = e->eng->budget();
    return IM_OK;
}

im_status im_engine_set_tuning(im_engine* e, const im_tuning* t)
{
    if (!e || !t) return imx::set_error(IM_EINVAL, "NULL argument");
    return e->eng->set_tuning(*t);
}

im_status im_engine_get_tuning(const im_engine* e, im_tuning* t)
{
    if (!e || !t) return imx::set_error(IM_EINVAL, "NULL argument");
    *t = e->eng->tuning();
    return IM_OK;
}

im_status im_engine_counters(const im_engine* e, int64_t* steps, int64_t* graphs_built, int64_t* graph_replays)
{
    if (!e) return imx::set_error(IM_EINVAL, "engine is NULL");
    e->eng->counters(steps, graphs_built, graph_replays);
    return IM_OK;
}

uint64_t im_query_footprint(const im_graph* g, int32_t J, int32_t K)
{
    if (!g || J < 64 || J > imx::kMaxJ || K < 1) return 0;
    return Engine::footprint(g, J, K);
}

void im_engine_free(im_engine* e)
{
    if (!e) return;
    for (Query* q : e->queries) e->eng->destroy(q);
    delete e;
}

im_status im_select_seeds_batch(int32_t G, const im_graph* const* graphs, const int32_t* J, const uint64_t* seed,
                                const int32_t* K, int32_t* const* seeds_out, double* spread_out, void* stream)
{
    if (G < 1 || !graphs || !J || !seed || !K || !seeds_out) return imx::set_error(IM_EINVAL, "NULL argument");
    im_engine* e = nullptr;
    if (im_status st = im_engine_create(G, 0, stream, &e)) return st;
    // many queries of one call (16 or more): captured steps with device-side
    // splits (the launch sequence changes only when a query finishes).  Fewer
    // queries use direct launches: a captured step launches every kernel kind
    // every round, which few queries cannot fill (one large query: 46% slower).
    im_tuning t = e->eng->tuning();
    t.use_graphs = G >= 16 ? 1 : 0;
    if (im_status st = e->eng->set_tuning(t)) {
        im_engine_free(e);
        return st;
    }
    std::vector<int64_t> ids(G);
    for (int32_t i = 0; i < G; ++i)
        if (im_status st = im_engine_submit(e, graphs[i], J[i], seed[i], K[i], &ids[i])) {
            im_engine_free(e);
            return st;
        }
    if (im_status st = e->eng->run()) {
        im_engine_free(e);
        return st;
    }
    for (int32_t i = 0; i < G; ++i)
        if (im_status st = im_engine_result(e, ids[i], seeds_out[i], spread_out ? &spread_out[i] : nullptr, nullptr,
                                            nullptr, nullptr)) {
            im_engine_free(e);
            return st;
        }
    im_engine_free(e);
    return IM_OK;
}

}  // extern "C"
