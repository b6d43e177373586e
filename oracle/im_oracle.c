/*
 * im_oracle.c -- plain, slow CPU reference of the sketch-based influence-
 * maximisation method (DiFuseR).  TEST INFRASTRUCTURE ONLY: tests, the smoke
 * check and the benchmark's CPU-baseline leg call it; the product path never
 * does.  It shares no code with the HIP library.
 *
 * Every step is written in the paper's order with plain loops, one simulation
 * (register index j) at a time where the paper works per simulation:
 *   - edge hash h(u,v)                      Section 2.2, Eq. 1
 *   - live test  (X_j xor h) < w            Section 2.2, Eq. 2 (fixed point form)
 *   - sketch init M_u[j] = rank_j(u)        Section 2.3, Eq. 3; Alg. 1 (Fill-Sketches)
 *   - union / add = register max            Section 2.3, Eq. 4-5
 *   - one synchronous sweep of pulls        Section 3.2, Alg. 2 (Simulate)
 *   - harmonic-mean cardinality estimate    Section 3.1, Eq. 7
 *   - greedy driver with cascade and the
 *     error-adaptive rebuild test           Section 4, Alg. 4; Section 3.3, Alg. 3
 *
 * Readings where the paper is silent (all stated in the project's design notes):
 *   hash      = MurmurHash3_x86_32 (Appleby), key LE32(u)||LE32(v), seed 0, & 0x7fffffff
 *   X         = top 31 bits of SplitMix64 outputs 0..J-1 for the build seed, sorted
 *   threshold = W = min(2^31, floor(p_float32 * 2^31)); live iff (X xor h) < W
 *   rank      = clz32(Murmur3(LE32(seed_lo)||LE32(seed_hi)||LE32(u)||LE32(j), 1)) + 1
 *   covered registers are stored as 0; the oracle also keeps the covered sets
 *   explicitly (cov[u*J+j]) and never infers coverage from register values.
 *   estimate  = alpha_J * 2^33 * J_u^2 / (J * H_u), with J_u = #uncovered
 *               registers and H_u = sum over uncovered j of 2^(33 - M[u][j])
 *   argmax    = exact rational compare of J_u^2/H_u, lowest id on ties, seeds
 *               excluded; a vertex with J_u = 0 has value 0
 *   rebuild   = after pick k < K, if 100*(T - T_old) > T (T = covered pairs)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

/* ------------------------------------------------------------------ hashing */

static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

/* MurmurHash3_x86_32 as published by Austin Appleby (public domain algorithm):
 * 4-byte little-endian blocks, tail bytes, length xor and the fmix32 finaliser. */
uint32_t orc_murmur3_32(const uint8_t* key, int64_t len, uint32_t seed)
{
    const uint32_t c1 = 0xcc9e2d51u, c2 = 0x1b873593u;
    uint32_t h = seed;
    int64_t nblocks = len / 4;
    for (int64_t i = 0; i < nblocks; ++i) {
        uint32_t k = (uint32_t)key[4 * i] | ((uint32_t)key[4 * i + 1] << 8) |
                     ((uint32_t)key[4 * i + 2] << 16) | ((uint32_t)key[4 * i + 3] << 24);
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
        h = rotl32(h, 13);
        h = h * 5u + 0xe6546b64u;
    }
    const uint8_t* tail = key + nblocks * 4;
    uint32_t k1 = 0;
    switch (len & 3) {
    case 3: k1 ^= (uint32_t)tail[2] << 16; /* fall through */
    case 2: k1 ^= (uint32_t)tail[1] << 8;  /* fall through */
    case 1:
        k1 ^= tail[0];
        k1 *= c1;
        k1 = rotl32(k1, 15);
        k1 *= c2;
        h ^= k1;
    }
    h ^= (uint32_t)len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

static void put_le32(uint8_t* b, uint32_t x)
{
    b[0] = (uint8_t)x; b[1] = (uint8_t)(x >> 8); b[2] = (uint8_t)(x >> 16); b[3] = (uint8_t)(x >> 24);
}

/* SplitMix64 (Steele, Lea, Flood 2014): state advances by the golden gamma,
 * output is the variant-13 mix of the state.  Returns output number i (i >= 0)
 * of the stream started at `seed`. */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* Eq. 1: h(u,v) = Murmur3(u || v) mod 2^31. */
uint32_t orc_edge_hash(uint32_t u, uint32_t v)
{
    uint8_t key[8];
    put_le32(key, u);
    put_le32(key + 4, v);
    return orc_murmur3_32(key, 8, 0u) & 0x7fffffffu;
}

/* Eq. 3 with the HyperLogLog offset: rank = leading zeros of the j-th hash of u, plus one. */
static int clz32(uint32_t x)
{
    int c = 0;
    if (x == 0) return 32;
    while (!(x & 0x80000000u)) { x <<= 1; ++c; }
    return c;
}

uint8_t orc_rank(uint64_t seed, uint32_t u, uint32_t j)
{
    uint8_t key[16];
    put_le32(key, (uint32_t)seed);
    put_le32(key + 4, (uint32_t)(seed >> 32));
    put_le32(key + 8, u);
    put_le32(key + 12, j);
    return (uint8_t)(clz32(orc_murmur3_32(key, 16, 1u)) + 1);
}

/* Fixed-point edge threshold from the float32 probability (Section 4.1 states
 * that P and w use a fixed-point representation). */
uint32_t orc_threshold(float p)
{
    double w = (double)p * 2147483648.0;
    if (w >= 2147483648.0) return 0x80000000u;
    if (w <= 0.0) return 0u;
    return (uint32_t)w; /* truncation == floor for positive values */
}

/* Eq. 2: edge live in simulation j iff (X_j xor h) / h_max < w, i.e. (X_j xor h) < W. */
int orc_live(uint32_t X, uint32_t h, uint32_t W) { return (X ^ h) < W; }

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/* Random values X_1..X_J of the simulations, sorted ascending (Section 4.1). */
void orc_sim_values(uint64_t seed, int32_t J, uint32_t* X)
{
    for (int32_t i = 0; i < J; ++i) X[i] = (uint32_t)(orc_splitmix64_at(seed, (uint64_t)i) >> 33);
    qsort(X, (size_t)J, sizeof(uint32_t), cmp_u32);
}

/* HyperLogLog bias constant alpha_J (Flajolet, Fusy, Gandouet, Meunier 2007). */
double orc_alpha(int32_t J)
{
    if (J == 16) return 0.673;
    if (J == 32) return 0.697;
    if (J == 64) return 0.709;
    return 0.7213 / (1.0 + 1.079 / (double)J);
}

/* ------------------------------------------------------------------ graph helpers */

typedef struct {
    int64_t n, m;
    const int64_t* rowptr;
    const int32_t* col;
    uint32_t* h;  /* per-edge hash, Eq. 1 */
    uint32_t* W;  /* per-edge threshold */
} orc_graph;

static int graph_init(orc_graph* g, int64_t n, const int64_t* rowptr, const int32_t* col, const float* p)
{
    g->n = n;
    g->m = rowptr[n];
    g->rowptr = rowptr;
    g->col = col;
    g->h = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(g->m ? g->m : 1));
    g->W = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(g->m ? g->m : 1));
    if (!g->h || !g->W) { free(g->h); free(g->W); return ORC_ENOMEM; }
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            g->h[e] = orc_edge_hash((uint32_t)u, (uint32_t)col[e]);
            g->W[e] = orc_threshold(p[e]);
        }
    return ORC_OK;
}

static void graph_free(orc_graph* g) { free(g->h); free(g->W); }

/* ------------------------------------------------------------------ Alg. 1 and Alg. 2 */

/* Alg. 1 (Fill-Sketches): every uncovered register is reset to the vertex's own
 * rank; covered registers stay 0. */
void orc_fill(int64_t n, int32_t J, uint64_t seed, const uint8_t* cov, uint8_t* M)
{
    for (int64_t u = 0; u < n; ++u)
        for (int32_t j = 0; j < J; ++j) {
            size_t i = (size_t)u * (size_t)J + (size_t)j;
            M[i] = (cov && cov[i]) ? 0 : orc_rank(seed, (uint32_t)u, (uint32_t)j);
        }
}

/* Alg. 2 (Simulate), one synchronous sweep: for every uncovered (u, j),
 * Mn[u][j] = max(M[u][j], max over out-edges (u,v) live in j of M[v][j]).
 * Returns the number of registers that changed. */
static int64_t simulate_sweep(const orc_graph* g, int32_t J, const uint32_t* X, const uint8_t* cov,
                              const uint8_t* M, uint8_t* Mn)
{
    int64_t changed = 0;
    for (int64_t u = 0; u < g->n; ++u) {
        for (int32_t j = 0; j < J; ++j) {
            size_t iu = (size_t)u * (size_t)J + (size_t)j;
            uint8_t best = M[iu];
            if (!(cov && cov[iu])) {
                for (int64_t e = g->rowptr[u]; e < g->rowptr[u + 1]; ++e) {
                    if (!orc_live(X[j], g->h[e], g->W[e])) continue;
                    uint8_t mv = M[(size_t)g->col[e] * (size_t)J + (size_t)j];
                    if (mv > best) best = mv;
                }
            }
            if (best != M[iu]) ++changed;
            Mn[iu] = best;
        }
    }
    return changed;
}

/* Build = Fill then Simulate sweeps until a sweep changes nothing.  The sweep
 * count includes that final no-change sweep. */
static int build(const orc_graph* g, int32_t J, uint64_t seed, const uint32_t* X, const uint8_t* cov,
                 uint8_t* M, uint8_t* tmp, int32_t* sweeps)
{
    orc_fill(g->n, J, seed, cov, M);
    int32_t it = 0;
    for (;;) {
        int64_t ch = simulate_sweep(g, J, X, cov, M, tmp);
        ++it;
        memcpy(M, tmp, (size_t)g->n * (size_t)J);
        if (ch == 0) break;
    }
    if (sweeps) *sweeps = it;
    return ORC_OK;
}

/* Public: build registers of a fresh sketch (nothing covered). */
int orc_build(int64_t n, const int64_t* rowptr, const int32_t* col, const float* p, int32_t J, uint64_t seed,
              uint8_t* M_out, int32_t* sweeps_out)
{
    if (n < 0 || J <= 0) return ORC_EINVAL;
    orc_graph g;
    int st = graph_init(&g, n, rowptr, col, p);
    if (st) return st;
    uint32_t* X = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)J);
    uint8_t* tmp = (uint8_t*)malloc((size_t)(n ? n : 1) * (size_t)J);
    if (!X || !tmp) { free(X); free(tmp); graph_free(&g); return ORC_ENOMEM; }
    orc_sim_values(seed, J, X);
    build(&g, J, seed, X, NULL, M_out, tmp, sweeps_out);
    free(X); free(tmp); graph_free(&g);
    return ORC_OK;
}

/* Run `nsweeps` synchronous sweeps of Alg. 2 for a subset of simulations only
 * (columns sims[0..S-1] of a J-wide sketch, nothing covered) starting from
 * Fill (Alg. 1); used to time the oracle on a bounded sample of a large
 * workload.  Returns the number of registers the last sweep changed in
 * *last_changed and, when M_out is not NULL, the registers after the last
 * sweep as uint8[n][S] (column s is simulation sims[s]). */
int orc_sweeps_sample(int64_t n, const int64_t* rowptr, const int32_t* col, const float* p, int32_t J,
                      uint64_t seed, const int32_t* sims, int32_t S, int32_t nsweeps, int64_t* last_changed,
                      uint8_t* M_out)
{
    orc_graph g;
    int st = graph_init(&g, n, rowptr, col, p);
    if (st) return st;
    uint32_t* X = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)J);
    uint32_t* Xs = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)S);
    uint8_t* M = (uint8_t*)malloc((size_t)(n ? n : 1) * (size_t)S);
    uint8_t* Mn = (uint8_t*)malloc((size_t)(n ? n : 1) * (size_t)S);
    if (!X || !Xs || !M || !Mn) { free(X); free(Xs); free(M); free(Mn); graph_free(&g); return ORC_ENOMEM; }
    orc_sim_values(seed, J, X);
    for (int32_t s = 0; s < S; ++s) Xs[s] = X[sims[s]];
    for (int64_t u = 0; u < n; ++u)
        for (int32_t s = 0; s < S; ++s) M[(size_t)u * S + s] = orc_rank(seed, (uint32_t)u, (uint32_t)sims[s]);
    int64_t ch = 0;
    for (int32_t it = 0; it < nsweeps; ++it) {
        ch = simulate_sweep(&g, S, Xs, NULL, M, Mn);
        memcpy(M, Mn, (size_t)n * (size_t)S);
    }
    if (last_changed) *last_changed = ch;
    if (M_out) memcpy(M_out, M, (size_t)n * (size_t)S);
    free(X); free(Xs); free(M); free(Mn); graph_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------ estimate and argmax */

/* Per vertex: J_u = number of uncovered registers, H_u = sum of 2^(33 - M) over them. */
void orc_estimates(int64_t n, int32_t J, const uint8_t* M, const uint8_t* cov, uint32_t* Ju, uint64_t* Hu)
{
    for (int64_t u = 0; u < n; ++u) {
        uint32_t c = 0;
        uint64_t h = 0;
        for (int32_t j = 0; j < J; ++j) {
            size_t i = (size_t)u * (size_t)J + (size_t)j;
            int covered = cov ? cov[i] : (M[i] == 0);
            if (covered) continue;
            ++c;
            h += (uint64_t)1 << (33 - M[i]);
        }
        Ju[u] = c;
        Hu[u] = h;
    }
}

/* Does vertex a have a strictly larger value J_a^2/H_a than b?  Value is 0 when J = 0. */
static int value_greater(uint32_t Ja, uint64_t Ha, uint32_t Jb, uint64_t Hb)
{
    if (Ja == 0) return 0;
    if (Jb == 0) return 1;
    unsigned __int128 lhs = (unsigned __int128)((uint64_t)Ja * Ja) * Hb;
    unsigned __int128 rhs = (unsigned __int128)((uint64_t)Jb * Jb) * Ha;
    return lhs > rhs;
}

int64_t orc_argmax(int64_t n, const uint32_t* Ju, const uint64_t* Hu, const uint8_t* is_seed)
{
    int64_t best = -1;
    for (int64_t u = 0; u < n; ++u) {
        if (is_seed && is_seed[u]) continue;
        if (best < 0 || value_greater(Ju[u], Hu[u], Ju[best], Hu[best])) best = u;
    }
    return best;
}

double orc_estimate_value(int32_t J, uint32_t Js, uint64_t Hs)
{
    if (Js == 0) return 0.0;
    double a = orc_alpha(J) * 8589934592.0;
    double q = (double)((uint64_t)Js * Js) / ((double)J * (double)Hs);
    return a * q;
}

/* ------------------------------------------------------------------ cascade (Alg. 3 result) */

/* Cover everything reachable from s in simulation j through live edges:
 * C_j <- C_j  union  R_j(s).  Plain BFS per simulation.  Returns #newly covered. */
static int64_t cascade_one_sim(const orc_graph* g, int32_t J, const uint32_t* X, int32_t j, int64_t s,
                               uint8_t* cov, int32_t* queue)
{
    size_t is = (size_t)s * (size_t)J + (size_t)j;
    if (cov[is]) return 0;
    int64_t head = 0, tail = 0, added = 0;
    cov[is] = 1;
    ++added;
    queue[tail++] = (int32_t)s;
    while (head < tail) {
        int64_t x = queue[head++];
        for (int64_t e = g->rowptr[x]; e < g->rowptr[x + 1]; ++e) {
            if (!orc_live(X[j], g->h[e], g->W[e])) continue;
            int64_t y = g->col[e];
            size_t iy = (size_t)y * (size_t)J + (size_t)j;
            if (cov[iy]) continue;
            cov[iy] = 1;
            ++added;
            queue[tail++] = (int32_t)y;
        }
    }
    return added;
}

/* ------------------------------------------------------------------ Alg. 4 driver */

/*
 * Greedy seed selection on one device (mu = 1): build, then K times
 * estimate -> argmax -> cascade -> score -> maybe rebuild.
 * Optional outputs (NULL to skip):
 *   seeds[K], est[K] (estimate of each pick), T[K] (covered pairs after each
 *   cascade), sweeps[K] (sweeps of the initial build in sweeps[0]; sweeps[k]
 *   for k >= 1 is the sweep count of the rebuild done just before pick k, 0
 *   when there was none), M_build0[n*J]
 *   (registers after the initial build), Ju0[n], Hu0[n] (estimates before
 *   the first pick), M_final[n*J] (registers at the end), spread (T_K / J).
 */
int orc_greedy(int64_t n, const int64_t* rowptr, const int32_t* col, const float* p, int32_t J, uint64_t seed,
               int32_t K, int32_t* seeds, double* est, uint64_t* T, int32_t* sweeps, uint8_t* M_build0,
               uint32_t* Ju0, uint64_t* Hu0, uint8_t* M_final, double* spread)
{
    if (n <= 0 || J <= 0 || K < 1 || K > n) return ORC_EINVAL;
    orc_graph g;
    int st = graph_init(&g, n, rowptr, col, p);
    if (st) return st;
    size_t nJ = (size_t)n * (size_t)J;
    uint32_t* X = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)J);
    uint8_t* M = (uint8_t*)malloc(nJ);
    uint8_t* tmp = (uint8_t*)malloc(nJ);
    uint8_t* cov = (uint8_t*)calloc(nJ, 1);
    uint8_t* is_seed = (uint8_t*)calloc((size_t)n, 1);
    uint32_t* Ju = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    uint64_t* Hu = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!X || !M || !tmp || !cov || !is_seed || !Ju || !Hu || !queue) {
        st = ORC_ENOMEM;
        goto done;
    }
    orc_sim_values(seed, J, X);

    int32_t sw = 0;
    build(&g, J, seed, X, cov, M, tmp, &sw);
    if (sweeps) sweeps[0] = sw;
    if (M_build0) memcpy(M_build0, M, nJ);

    uint64_t score = 0, oldscore = 0;
    for (int32_t k = 0; k < K; ++k) {
        orc_estimates(n, J, M, cov, Ju, Hu);
        if (k == 0 && Ju0) memcpy(Ju0, Ju, sizeof(uint32_t) * (size_t)n);
        if (k == 0 && Hu0) memcpy(Hu0, Hu, sizeof(uint64_t) * (size_t)n);
        int64_t s = orc_argmax(n, Ju, Hu, is_seed);
        is_seed[s] = 1;
        if (seeds) seeds[k] = (int32_t)s;
        if (est) est[k] = orc_estimate_value(J, Ju[s], Hu[s]);

        for (int32_t j = 0; j < J; ++j) score += (uint64_t)cascade_one_sim(&g, J, X, j, s, cov, queue);
        for (size_t i = 0; i < nJ; ++i)
            if (cov[i]) M[i] = 0;
        if (T) T[k] = score;

        if (k + 1 < K) {
            int32_t rs = 0;
            if (100 * (score - oldscore) > score) {
                build(&g, J, seed, X, cov, M, tmp, &rs);
                oldscore = score;
            }
            if (sweeps) sweeps[k + 1] = rs;
        }
    }
    if (M_final) memcpy(M_final, M, nJ);
    if (spread) *spread = (double)score / (double)J;

done:
    free(X); free(M); free(tmp); free(cov); free(is_seed); free(Ju); free(Hu); free(queue);
    graph_free(&g);
    return st;
}

/* ------------------------------------------------------------------ closed forms used as pins */

/* Per-arc hash (Eq. 1) and fixed-point threshold for a whole CSR graph. */
void orc_graph_hashes(int64_t n, const int64_t* rowptr, const int32_t* col, const float* p, uint32_t* h, uint32_t* W)
{
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            h[e] = orc_edge_hash((uint32_t)u, (uint32_t)col[e]);
            W[e] = orc_threshold(p[e]);
        }
}

/* Fixed point of Alg. 2 in closed form: the register of an uncovered vertex u
 * in simulation j is the largest rank over the vertices reachable from u in the
 * live graph of simulation j without entering covered vertices (covered
 * registers are 0 and the covered set is closed under live arcs).  Returns 0
 * when u itself is covered.  covered_j: n flags for simulation j, or NULL. */
int orc_reach_max(int64_t n, const int64_t* rowptr, const int32_t* col, const uint32_t* h, const uint32_t* W,
                  uint32_t Xj, uint64_t seed, int32_t j, int64_t u, const uint8_t* covered_j)
{
    if (covered_j && covered_j[u]) return 0;
    uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!seen || !queue) { free(seen); free(queue); return -1; }
    int64_t head = 0, tail = 0;
    int best = 0;
    seen[u] = 1;
    queue[tail++] = (int32_t)u;
    while (head < tail) {
        int64_t x = queue[head++];
        int r = orc_rank(seed, (uint32_t)x, (uint32_t)j);
        if (r > best) best = r;
        for (int64_t e = rowptr[x]; e < rowptr[x + 1]; ++e) {
            int64_t y = col[e];
            if (seen[y] || !orc_live(Xj, h[e], W[e])) continue;
            if (covered_j && covered_j[y]) continue;
            seen[y] = 1;
            queue[tail++] = (int32_t)y;
        }
    }
    free(seen);
    free(queue);
    return best;
}

/* Covered set of simulation j for a seed set: union of the live-graph
 * reachability sets of the sources (cascade result).  Writes n flags and
 * returns the number of covered vertices. */
int64_t orc_cover_from(int64_t n, const int64_t* rowptr, const int32_t* col, const uint32_t* h, const uint32_t* W,
                       uint32_t Xj, const int32_t* sources, int64_t nsrc, uint8_t* covered_out)
{
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    if (!queue) return -1;
    memset(covered_out, 0, (size_t)n);
    int64_t head = 0, tail = 0;
    for (int64_t i = 0; i < nsrc; ++i) {
        int64_t s = sources[i];
        if (covered_out[s]) continue;
        covered_out[s] = 1;
        queue[tail++] = (int32_t)s;
    }
    while (head < tail) {
        int64_t x = queue[head++];
        for (int64_t e = rowptr[x]; e < rowptr[x + 1]; ++e) {
            int64_t y = col[e];
            if (covered_out[y] || !orc_live(Xj, h[e], W[e])) continue;
            covered_out[y] = 1;
            queue[tail++] = (int32_t)y;
        }
    }
    free(queue);
    return tail;
}
