/*
 * felog_oracle.c -- plain, slow CPU oracle for the FeLoG hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load this file's library.  It shares no code, header,
 * table or constant generator with the HIP library, and the HIP library never
 * calls it.
 *
 * What it computes, and where the paper defines it:
 *   - truncated uniform random walks (DeepWalk), Section 2 "Sampling process";
 *   - second-order node2vec walks, named in Sections 3 and 5.4 (the paper gives
 *     no formula; the original node2vec bias with return parameter p and in-out
 *     parameter q is used, drawn by rejection);
 *   - skip-gram with negative sampling, Eq. (1) and Eq. (2), with the sigmoid
 *     defined right after Table 1, updated by plain SGD on the negated Eq. (2)
 *     objective;
 *   - the neighbourhood-consistency score Psi of Eq. (4) over a subsampled
 *     neighbourhood, and the active-set rule of Eq. (5) (Algorithm 1 runs them
 *     in a loop; the loop itself is in oracle/__init__.py).
 *
 * Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 * written here from its published definition.  Every floating-point value the
 * method produces is computed in double precision unless it is an FP32 table
 * entry; comparisons that decide an integer (node2vec acceptance) use the FP32
 * operations that define them.
 *
 * Loops over independent items (table rows, walks, scored nodes, the
 * coefficients of a minibatch's pairs) run under OpenMP; every value is
 * computed as in a one-thread run, and every sum keeps its order, so the
 * results do not depend on the number of threads.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared -ffp-contract=off -fno-fast-math
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the OpenMP loops (for the CPU-baseline timings). */
void orc_set_threads(int k) { omp_set_num_threads(k > 0 ? k : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Philox4x32-10, SC'11: multipliers and Weyl key increments.          */
/* ------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

/* Stream tags, placed in the top byte of counter word 3. */
enum { TAG_WALK = 1, TAG_N2V = 2, TAG_NEG = 3, TAG_INIT = 4, TAG_PSI = 5,
       TAG_SHNEG = 6 };

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t q = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(q >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)q;
        uint32_t y2 = (uint32_t)(p >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_WEYL_A;
        k1 += PHILOX_WEYL_B;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_u64key(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                          uint64_t seed, uint32_t out[4])
{
    uint32_t ctr[4] = { c0, c1, c2, c3 };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox(ctr, key, out);
}

/* Uniform integer in [0, m) from one 32-bit draw: floor(x * m / 2^32). */
static inline uint32_t below32(uint32_t x, uint32_t m)
{
    return (uint32_t)(((uint64_t)x * (uint64_t)m) >> 32);
}

void orc_philox_batch(int64_t count, const uint32_t* ctrs, uint64_t seed, uint32_t* outs)
{
    for (int64_t i = 0; i < count; ++i)
        philox_u64key(ctrs[4 * i], ctrs[4 * i + 1], ctrs[4 * i + 2], ctrs[4 * i + 3],
                      seed, outs + 4 * i);
}

/* ------------------------------------------------------------------ */
/* Embedding initialisation: in ~ U(-0.5/d, 0.5/d), out = 0.           */
/* ------------------------------------------------------------------ */
void orc_init_tables(int64_t n, int d, uint64_t seed, float* in, float* out)
{
    /* rows are independent; one Philox call serves columns 4m .. 4m+3 */
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
        uint32_t r[4];
        for (int c = 0; c < d; ++c) {
            if (c % 4 == 0)
                philox_u64key((uint32_t)v, (uint32_t)(v >> 32), (uint32_t)(c / 4),
                              (uint32_t)TAG_INIT << 24, seed, r);
            float u = (float)(r[c % 4] >> 8) * (1.0f / 16777216.0f);  /* [0,1), 24 bits */
            in[v * d + c] = (u - 0.5f) / (float)d;
            out[v * d + c] = 0.0f;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Noise distribution Pn(u) proportional to count^0.75.                */
/* Weight of node i: floor(2^16 * sqrt(c) * sqrt(sqrt(c))) in IEEE     */
/* double arithmetic; draws use the exact integer inverse CDF.         */
/* ------------------------------------------------------------------ */
void orc_neg_weights(int64_t n, const uint64_t* counts, uint64_t* w)
{
    for (int64_t i = 0; i < n; ++i) {
        double c = (double)counts[i];
        double s = sqrt(c);
        double t = sqrt(s);
        double x = s * t;                /* c^(3/4) */
        w[i] = (uint64_t)(x * 65536.0);  /* exact scaling, then truncation */
    }
}

void orc_cdf(int64_t n, const uint64_t* w, uint64_t* cdf)
{
    cdf[0] = 0;
    for (int64_t i = 0; i < n; ++i) cdf[i + 1] = cdf[i] + w[i];
}

/* Smallest i with cdf[i+1] > u, where u = floor(x * T / 2^64). */
int32_t orc_inverse_cdf(int64_t n, const uint64_t* cdf, uint64_t x)
{
    uint64_t T = cdf[n];
    uint64_t u = (uint64_t)(((unsigned __int128)x * (unsigned __int128)T) >> 64);
    int64_t lo = 0, hi = n - 1;           /* answer in [lo, hi] */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
    }
    return (int32_t)lo;
}

void orc_draw_batch(int64_t n, const uint64_t* cdf, int64_t count, const uint64_t* xs, int32_t* out)
{
    for (int64_t i = 0; i < count; ++i) out[i] = orc_inverse_cdf(n, cdf, xs[i]);
}

/* ------------------------------------------------------------------ */
/* Walks.  L counts nodes including the start; a start node with no     */
/* neighbours gives a one-node walk padded with -1.  Walk number wi of    */
/* the call has id id_base + wi and starts at starts[wi % n_starts].     */
/* Output is walk-major [W][L].                                          */
/* ------------------------------------------------------------------ */
void orc_walks_uniform(int64_t n, const int64_t* indptr, const int32_t* indices,
                       const int32_t* starts, int64_t n_starts, int r, int L,
                       uint64_t seed, int64_t id_base, int32_t* walks)
{
    (void)n;
    int64_t W = n_starts * (int64_t)r;
    /* walks are independent */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t wi = 0; wi < W; ++wi) {
        int32_t* out = walks + wi * L;
        int64_t wid = id_base + wi;
        int32_t v = starts[wi % n_starts];
        out[0] = v;
        int t;
        for (t = 0; t + 1 < L; ++t) {
            int64_t deg = indptr[v + 1] - indptr[v];
            if (deg == 0) break;
            uint32_t x[4];
            philox_u64key((uint32_t)wid, (uint32_t)(wid >> 32), (uint32_t)t,
                          (uint32_t)TAG_WALK << 24, seed, x);
            v = indices[indptr[v] + below32(x[0], (uint32_t)deg)];
            out[t + 1] = v;
        }
        for (int s = t + 1; s < L; ++s) out[s] = -1;
    }
}

static int is_neighbour(const int64_t* indptr, const int32_t* indices, int32_t a, int32_t b)
{
    int64_t lo = indptr[a], hi = indptr[a + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (indices[mid] < b) lo = mid + 1; else hi = mid;
    }
    return lo < indptr[a + 1] && indices[lo] == b;
}

/*
 * Second-order walk.  From current node v with previous node t, the next node x
 * has probability proportional to w(v,x) * alpha(t,x) with alpha = 1/p if x == t,
 * 1 if x is a neighbour of t, 1/q otherwise; the first transition uses alpha = 1.
 * Draw by rejection: propose x uniformly among v's neighbours, accept when
 * u * (wmax(v) * alpha_max) < w(v,x) * alpha(t,x) in FP32, with u in [0,1) of 24
 * bits.  After max_attempts rejections the last proposal is taken (counted).
 */
int64_t orc_walks_node2vec(int64_t n, const int64_t* indptr, const int32_t* indices,
                           const float* weights, const int32_t* starts, int64_t n_starts,
                           int r, int L, float p, float q, int max_attempts,
                           uint64_t seed, int64_t id_base, int32_t* walks)
{
    float inv_p = 1.0f / p, inv_q = 1.0f / q;
    float amax = 1.0f;
    if (inv_p > amax) amax = inv_p;
    if (inv_q > amax) amax = inv_q;
    float* wmax = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    for (int64_t v = 0; v < n; ++v) {
        float m = 0.0f;
        for (int64_t e = indptr[v]; e < indptr[v + 1]; ++e) {
            float w = weights ? weights[e] : 1.0f;
            if (w > m) m = w;
        }
        wmax[v] = m;
    }
    int64_t capped = 0;
    int64_t W = n_starts * (int64_t)r;
    /* walks are independent */
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : capped)
    for (int64_t wi = 0; wi < W; ++wi) {
        int32_t* out = walks + wi * L;
        int64_t wid = id_base + wi;
        int32_t v = starts[wi % n_starts];
        int32_t prev = -1;
        out[0] = v;
        int t;
        for (t = 0; t + 1 < L; ++t) {
            int64_t deg = indptr[v + 1] - indptr[v];
            if (deg == 0) break;
            int32_t x = -1;
            for (int a = 0; a < max_attempts; ++a) {
                uint32_t rr[4];
                philox_u64key((uint32_t)wid, (uint32_t)(wid >> 32), (uint32_t)t,
                              ((uint32_t)TAG_N2V << 24) | (uint32_t)a, seed, rr);
                int64_t e = indptr[v] + below32(rr[0], (uint32_t)deg);
                x = indices[e];
                float w = weights ? weights[e] : 1.0f;
                float u = (float)(rr[1] >> 8) * (1.0f / 16777216.0f);
                float alpha, bound;
                if (t == 0) {
                    alpha = 1.0f;
                    bound = wmax[v];
                } else {
                    if (x == prev) alpha = inv_p;
                    else if (is_neighbour(indptr, indices, prev, x)) alpha = 1.0f;
                    else alpha = inv_q;
                    bound = wmax[v] * amax;
                }
                float lhs = u * bound;
                float rhs = w * alpha;
                if (lhs < rhs) break;
                if (a == max_attempts - 1) ++capped;
            }
            prev = v;
            v = x;
            out[t + 1] = v;
        }
        for (int s = t + 1; s < L; ++s) out[s] = -1;
    }
    free(wmax);
    return capped;
}

/* ------------------------------------------------------------------ */
/* Skip-gram pairs.  Within a chunk of consecutive walks, pairs are        */
/* ordered by centre position j, then offset i in (-w..-1, 1..w), then     */
/* walk; a pair exists when both positions hold a node.  A minibatch is     */
/* the next P pairs of the chunk (the chunk's last one may be short).      */
/* Offset slot s in [0, 2w): i = s - w for s < w, else s - w + 1.           */
/* ------------------------------------------------------------------ */
static int slot_offset(int s, int w) { return s < w ? s - w : s - w + 1; }

/* Pairs of each (j, slot) slice of walks [c0, c1): both positions hold a node. */
void orc_slice_counts(const int32_t* walks, int64_t c0, int64_t c1, int L, int w,
                      int64_t* counts)
{
    for (int j = 0; j < L; ++j)
        for (int s = 0; s < 2 * w; ++s) {
            int jj = j + slot_offset(s, w);
            int64_t cnt = 0;
            if (jj >= 0 && jj < L)
                for (int64_t col = c0; col < c1; ++col)
                    if (walks[col * L + j] >= 0 && walks[col * L + jj] >= 0) ++cnt;
            counts[(int64_t)j * 2 * w + s] = cnt;
        }
}

static int64_t chunk_pairs(const int32_t* walks, int64_t c0, int64_t c1, int L, int w)
{
    int64_t* counts = (int64_t*)malloc(sizeof(int64_t) * (size_t)L * 2 * w);
    orc_slice_counts(walks, c0, c1, L, w, counts);
    int64_t cnt = 0;
    for (int64_t i = 0; i < (int64_t)L * 2 * w; ++i) cnt += counts[i];
    free(counts);
    return cnt;
}

/* Number of minibatches (and pairs) a corpus yields. */
int64_t orc_count_minibatches(const int32_t* walks, int64_t W, int L, int w,
                              int64_t P, int64_t chunk, int64_t* total_pairs)
{
    int64_t B = 0, tp = 0;
    for (int64_t c0 = 0; c0 < W; c0 += chunk) {
        int64_t c1 = c0 + chunk < W ? c0 + chunk : W;
        int64_t np = chunk_pairs(walks, c0, c1, L, w);
        tp += np;
        B += (np + P - 1) / P;
    }
    if (total_pairs) *total_pairs = tp;
    return B;
}

/*
 * Pairs number [lo, lo + P) of the chunk of walks [c0, c1), in pair order:
 * ctx = walk[j+i], ctr = walk[j], plus the walk column, centre position j and
 * offset slot, which key the negative draws.  ``counts`` holds the chunk's
 * slice counts (orc_slice_counts); whole slices before ``lo`` are skipped.
 */
int64_t orc_chunk_pairs_range(const int32_t* walks, int64_t c0, int64_t c1, int L, int w,
                              const int64_t* counts, int64_t lo, int64_t P,
                              int32_t* ctx, int32_t* ctr, int64_t* col_out,
                              int32_t* j_out, int32_t* slot_out)
{
    int64_t idx = 0, k = 0, hi = lo + P;
    for (int j = 0; j < L; ++j)
        for (int s = 0; s < 2 * w; ++s) {
            int64_t cnt = counts[(int64_t)j * 2 * w + s];
            if (idx + cnt <= lo) { idx += cnt; continue; }   /* slice wholly before lo */
            int jj = j + slot_offset(s, w);
            if (jj < 0 || jj >= L) continue;
            for (int64_t col = c0; col < c1; ++col) {
                int32_t a = walks[col * L + jj], c = walks[col * L + j];
                if (a < 0 || c < 0) continue;
                if (idx >= lo) {
                    ctx[k] = a; ctr[k] = c; col_out[k] = col;
                    j_out[k] = j; slot_out[k] = s; ++k;
                }
                ++idx;
                if (idx >= hi) return k;
            }
        }
    return k;
}

/* Pairs of minibatch b of the whole corpus (chunks in order, P pairs each). */
int64_t orc_minibatch_pairs(const int32_t* walks, int64_t W, int L, int w,
                            int64_t P, int64_t chunk, int64_t b,
                            int32_t* ctx, int32_t* ctr, int64_t* col_out,
                            int32_t* j_out, int32_t* slot_out)
{
    int64_t first = 0;
    int64_t* counts = (int64_t*)malloc(sizeof(int64_t) * (size_t)L * 2 * w);
    for (int64_t c0 = 0; c0 < W; c0 += chunk) {
        int64_t c1 = c0 + chunk < W ? c0 + chunk : W;
        orc_slice_counts(walks, c0, c1, L, w, counts);
        int64_t np = 0;
        for (int64_t i = 0; i < (int64_t)L * 2 * w; ++i) np += counts[i];
        int64_t nb = (np + P - 1) / P;
        if (b >= first + nb) { first += nb; continue; }
        int64_t k = orc_chunk_pairs_range(walks, c0, c1, L, w, counts, (b - first) * P, P,
                                          ctx, ctr, col_out, j_out, slot_out);
        free(counts);
        return k;
    }
    free(counts);
    return 0;
}

/* K negatives per pair: draw k uses Philox(wid, j<<8|slot, k/2) words 2(k%2), 2(k%2)+1. */
void orc_draw_negatives(int64_t np, const int64_t* wid, const int32_t* j, const int32_t* slot,
                        int K, uint64_t seed, int64_t n, const uint64_t* cdf, int32_t* neg)
{
    for (int64_t p = 0; p < np; ++p)
        for (int k = 0; k < K; ++k) {
            uint32_t r[4];
            philox_u64key((uint32_t)wid[p], (uint32_t)(wid[p] >> 32),
                          ((uint32_t)j[p] << 8) | (uint32_t)slot[p],
                          ((uint32_t)TAG_NEG << 24) | (uint32_t)(k / 2), seed, r);
            int m = k % 2;
            uint64_t x = ((uint64_t)r[2 * m + 1] << 32) | (uint64_t)r[2 * m];
            neg[p * K + k] = orc_inverse_cdf(n, cdf, x);
        }
}

/* log(sigmoid(x)) without overflow. */
double orc_log_sigmoid(double x)
{
    if (x >= 0.0) return -log1p(exp(-x));
    return x - log1p(exp(x));
}

double orc_sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/*
 * One SGD minibatch on Eq. (2), instantiated for FP32 tables (the method's
 * storage) and FP64 tables (used by the finite-difference pins).
 *
 * For pair p with context c, centre t0 and negatives t1..tK (all read from the
 * tables as they stand at the start of the minibatch):
 *   s_k = in[c] . out[t_k]
 *   g_0 = lr (1 - sigma(s_0)),  g_k = -lr sigma(s_k)   (g_k = 0 when t_k == t0)
 *   delta_in[c]   += sum_k g_k out[t_k]
 *   delta_out[t_k] += g_k in[c]
 * All deltas of the minibatch are summed (in pair order, then k order) and
 * then added to the tables.  The minibatch loss is
 *   sum_p -[log sigma(s_0) + sum_k log sigma(-s_k)].
 *
 * If apply == 0 the tables are left untouched and the summed deltas are
 * returned as (rows, values) lists; the lists hold each touched row once,
 * in order of first touch.
 */
#define SGNS_DEFINE(NAME, T)                                                        \
double NAME(T* in, T* out, int64_t n, int d, int64_t np,                            \
            const int32_t* ctx, const int32_t* ctr, const int32_t* neg, int K,      \
            double lr, int apply,                                                   \
            int32_t* rows_in, double* d_in, int64_t* n_in,                          \
            int32_t* rows_out, double* d_out, int64_t* n_out)                       \
{                                                                                   \
    int32_t* slot_in = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);               \
    int32_t* slot_out = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);              \
    for (int64_t i = 0; i < n; ++i) { slot_in[i] = -1; slot_out[i] = -1; }          \
    int64_t cap_in = np, cap_out = np * (K + 1);                                    \
    int own = 0;                                                                    \
    if (!rows_in) {                                                                 \
        own = 1;                                                                    \
        rows_in = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap_in);              \
        d_in = (double*)malloc(sizeof(double) * (size_t)cap_in * d);               \
        rows_out = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap_out);            \
        d_out = (double*)malloc(sizeof(double) * (size_t)cap_out * d);             \
    }                                                                               \
    int64_t ui = 0, uo = 0;                                                         \
    double loss = 0.0;                                                              \
    /* coefficients and loss terms of every pair, from the tables at the start:    \
       pairs are independent here */                                                \
    double* gall = (double*)malloc(sizeof(double) * (size_t)(np * (K + 1) + 1));    \
    double* lall = (double*)malloc(sizeof(double) * (size_t)(np * (K + 1) + 1));    \
    _Pragma("omp parallel for schedule(static)")                                    \
    for (int64_t p = 0; p < np; ++p) {                                              \
        int32_t c = ctx[p];                                                         \
        for (int k = 0; k <= K; ++k) {                                              \
            int32_t t = k == 0 ? ctr[p] : neg[p * K + (k - 1)];                     \
            double* gk = gall + p * (K + 1) + k;                                    \
            double* lk = lall + p * (K + 1) + k;                                    \
            if (k > 0 && t == ctr[p]) { *gk = 0.0; *lk = 0.0; continue; }           \
            double s = 0.0;                                                         \
            for (int e = 0; e < d; ++e)                                             \
                s += (double)in[(int64_t)c * d + e] * (double)out[(int64_t)t * d + e]; \
            if (k == 0) { *gk = lr * (1.0 - orc_sigmoid(s)); *lk = orc_log_sigmoid(s); } \
            else { *gk = -lr * orc_sigmoid(s); *lk = orc_log_sigmoid(-s); }         \
        }                                                                           \
    }                                                                               \
    int32_t* tk = (int32_t*)malloc(sizeof(int32_t) * (size_t)(K + 1));             \
    for (int64_t p = 0; p < np; ++p) {                                              \
        int32_t c = ctx[p];                                                         \
        const double* g = gall + p * (K + 1);                                       \
        tk[0] = ctr[p];                                                             \
        for (int k = 1; k <= K; ++k) tk[k] = neg[p * K + (k - 1)];                  \
        for (int k = 0; k <= K; ++k) {                                              \
            if (k > 0 && tk[k] == tk[0]) continue;                                  \
            loss -= lall[p * (K + 1) + k];                                          \
        }                                                                           \
        if (slot_in[c] < 0) {                                                       \
            slot_in[c] = (int32_t)ui; rows_in[ui] = c;                              \
            memset(d_in + ui * d, 0, sizeof(double) * (size_t)d); ++ui;            \
        }                                                                           \
        double* di = d_in + (int64_t)slot_in[c] * d;                                \
        for (int k = 0; k <= K; ++k) {                                              \
            if (k > 0 && tk[k] == tk[0]) continue;                                  \
            int32_t t = tk[k];                                                      \
            for (int e = 0; e < d; ++e) di[e] += g[k] * (double)out[(int64_t)t * d + e]; \
        }                                                                           \
        for (int k = 0; k <= K; ++k) {                                              \
            if (k > 0 && tk[k] == tk[0]) continue;                                  \
            int32_t t = tk[k];                                                      \
            if (slot_out[t] < 0) {                                                  \
                slot_out[t] = (int32_t)uo; rows_out[uo] = t;                        \
                memset(d_out + uo * d, 0, sizeof(double) * (size_t)d); ++uo;       \
            }                                                                       \
            double* dd = d_out + (int64_t)slot_out[t] * d;                          \
            for (int e = 0; e < d; ++e) dd[e] += g[k] * (double)in[(int64_t)c * d + e]; \
        }                                                                           \
    }                                                                               \
    if (apply) {                                                                    \
        for (int64_t i = 0; i < ui; ++i)                                            \
            for (int e = 0; e < d; ++e) {                                           \
                T* x = &in[(int64_t)rows_in[i] * d + e];                            \
                *x = (T)((double)*x + d_in[i * d + e]);                             \
            }                                                                       \
        for (int64_t i = 0; i < uo; ++i)                                            \
            for (int e = 0; e < d; ++e) {                                           \
                T* x = &out[(int64_t)rows_out[i] * d + e];                          \
                *x = (T)((double)*x + d_out[i * d + e]);                            \
            }                                                                       \
    }                                                                               \
    if (n_in) *n_in = ui;                                                           \
    if (n_out) *n_out = uo;                                                         \
    if (own) { free(rows_in); free(d_in); free(rows_out); free(d_out); }            \
    free(gall); free(lall); free(tk); free(slot_in); free(slot_out);                \
    return loss;                                                                    \
}

SGNS_DEFINE(orc_sgns_step_f32, float)
SGNS_DEFINE(orc_sgns_step_f64, double)

/* Minibatch loss only (FP64 tables), used for finite differences. */
double orc_sgns_loss_f64(const double* in, const double* out, int d, int64_t np,
                         const int32_t* ctx, const int32_t* ctr, const int32_t* neg, int K)
{
    double loss = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        for (int k = 0; k <= K; ++k) {
            int32_t t = k == 0 ? ctr[p] : neg[p * K + k - 1];
            if (k > 0 && t == ctr[p]) continue;
            double s = 0.0;
            for (int e = 0; e < d; ++e)
                s += in[(int64_t)ctx[p] * d + e] * out[(int64_t)t * d + e];
            loss -= k == 0 ? orc_log_sigmoid(s) : orc_log_sigmoid(-s);
        }
    }
    return loss;
}

/* ------------------------------------------------------------------ */
/* Eq. (4): Psi(v) = mean over a neighbour subset of cos(in[v], in[u]).    */
/* The subset is all neighbours when deg(v) <= k_s, otherwise k_s distinct  */
/* neighbours chosen by Floyd's algorithm (Bentley & Floyd, CACM 1987) with */
/* draw m taken from Philox(v, round, m/4) word m%4.  Products and sums in  */
/* FP64.  A node without neighbours gets NaN (it is never active).         */
/* ------------------------------------------------------------------ */
static double cosine(const float* a, const float* b, int d)
{
    double dot = 0.0, na = 0.0, nb = 0.0;
    for (int e = 0; e < d; ++e) {
        dot += (double)a[e] * (double)b[e];
        na += (double)a[e] * (double)a[e];
        nb += (double)b[e] * (double)b[e];
    }
    if (na == 0.0 || nb == 0.0) return 0.0;
    return dot / (sqrt(na) * sqrt(nb));
}

int orc_neighbour_subset(const int64_t* indptr, int32_t v, int k_s, uint64_t seed,
                         uint32_t round, int64_t* pick)
{
    int64_t deg = indptr[v + 1] - indptr[v];
    if (deg <= k_s) {
        for (int64_t i = 0; i < deg; ++i) pick[i] = i;
        return (int)deg;
    }
    int cnt = 0;
    uint32_t r[4];
    for (int m = 0; m < k_s; ++m) {
        int64_t jj = deg - k_s + m;               /* Floyd: j from deg-k to deg-1 */
        if (m % 4 == 0)
            philox_u64key((uint32_t)v, round, (uint32_t)(m / 4), (uint32_t)TAG_PSI << 24, seed, r);
        int64_t t = below32(r[m % 4], (uint32_t)(jj + 1));   /* uniform in [0, jj] */
        int seen = 0;
        for (int i = 0; i < cnt; ++i) if (pick[i] == t) { seen = 1; break; }
        pick[cnt++] = seen ? jj : t;
    }
    return cnt;
}

void orc_psi(const float* in, int d, const int64_t* indptr, const int32_t* indices,
             const int32_t* nodes, int64_t count, int k_s, uint64_t seed, uint32_t round,
             double* psi)
{
    /* nodes are independent */
#pragma omp parallel
    {
        /* the subset never holds more than k_s entries */
        int64_t* pick = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k_s > 0 ? k_s : 1));
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < count; ++i) {
            int32_t v = nodes[i];
            int64_t deg = indptr[v + 1] - indptr[v];
            if (deg == 0) { psi[i] = NAN; continue; }
            int m = orc_neighbour_subset(indptr, v, k_s, seed, round, pick);
            double acc = 0.0;
            for (int j = 0; j < m; ++j) {
                int32_t u = indices[indptr[v] + pick[j]];
                acc += cosine(in + (int64_t)v * d, in + (int64_t)u * d, d);
            }
            psi[i] = acc / (double)m;
        }
        free(pick);
    }
}

/* ------------------------------------------------------------------ */
/* Shared-negative minibatch (the BF16 systems form).  P pairs share M      */
/* negatives; each (pair, negative) term carries weight K/M so that the      */
/* expected update equals Eq. (2) with K negatives per pair.  Terms whose     */
/* negative equals the pair's centre are dropped.  When bf16 != 0, table      */
/* rows are rounded to bfloat16 (round to nearest even) before use, and the   */
/* negative-term coefficients G are rounded to bfloat16 before the two         */
/* backward products, as the systems form does; all sums are FP64 here.       */
/* Deltas are returned densely for in[ctx] per pair slot and out rows.        */
/* ------------------------------------------------------------------ */
float orc_bf16_round(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) {         /* inf / nan */
        if (u & 0x007FFFFFu) u |= 0x00400000u;
        u &= 0xFFFF0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7FFFu + lsb;
        u &= 0xFFFF0000u;
    }
    float y;
    memcpy(&y, &u, 4);
    return y;
}

void orc_shared_neg_draw(int64_t b, uint32_t round, int M, uint64_t seed, int64_t n,
                         const uint64_t* cdf, int32_t* negs)
{
    for (int m = 0; m < M; ++m) {
        uint32_t r[4];
        philox_u64key((uint32_t)b, round, (uint32_t)(m / 2), (uint32_t)TAG_SHNEG << 24, seed, r);
        int h = m % 2;
        uint64_t x = ((uint64_t)r[2 * h + 1] << 32) | (uint64_t)r[2 * h];
        negs[m] = orc_inverse_cdf(n, cdf, x);
    }
}

/*
 * Inputs are FP32 master tables; outputs: dctx[P][d] (delta for in[ctx_p], one
 * per pair slot), dneg[M][d] (delta for out[neg_m], one per negative slot) and
 * dctr[P][d] (delta for out[ctr_p]).  Returns the minibatch loss
 *   sum_p -log sigma(s0_p) - (K/M) sum_{p,m} mask * log sigma(-S_pm).
 */
double orc_shared_neg_step(const float* in, const float* out, int d, int P, int M, int K,
                           const int32_t* ctx, const int32_t* ctr, const int32_t* neg,
                           double lr, int bf16, double* dctx, double* dneg, double* dctr)
{
    double* C = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* O = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* N = (double*)malloc(sizeof(double) * (size_t)M * d);
    double* G = (double*)malloc(sizeof(double) * (size_t)P * M);
    double loss = 0.0, wk = (double)K / (double)M;
    for (int p = 0; p < P; ++p)
        for (int e = 0; e < d; ++e) {
            float a = in[(int64_t)ctx[p] * d + e], o = out[(int64_t)ctr[p] * d + e];
            C[(int64_t)p * d + e] = bf16 ? orc_bf16_round(a) : a;
            O[(int64_t)p * d + e] = bf16 ? orc_bf16_round(o) : o;
        }
    for (int m = 0; m < M; ++m)
        for (int e = 0; e < d; ++e) {
            float x = out[(int64_t)neg[m] * d + e];
            N[(int64_t)m * d + e] = bf16 ? orc_bf16_round(x) : x;
        }
    for (int p = 0; p < P; ++p)
        for (int m = 0; m < M; ++m) {
            double s = 0.0;
            for (int e = 0; e < d; ++e) s += C[(int64_t)p * d + e] * N[(int64_t)m * d + e];
            double gv = 0.0;
            if (neg[m] != ctr[p]) {
                gv = -lr * wk * orc_sigmoid(s);
                loss -= wk * orc_log_sigmoid(-s);
                if (bf16) gv = (double)orc_bf16_round((float)gv);
            }
            G[(int64_t)p * M + m] = gv;
        }
    for (int p = 0; p < P; ++p) {
        double s0 = 0.0;
        for (int e = 0; e < d; ++e) s0 += C[(int64_t)p * d + e] * O[(int64_t)p * d + e];
        double g0 = lr * (1.0 - orc_sigmoid(s0));
        loss -= orc_log_sigmoid(s0);
        for (int e = 0; e < d; ++e) {
            double acc = g0 * O[(int64_t)p * d + e];
            for (int m = 0; m < M; ++m) acc += G[(int64_t)p * M + m] * N[(int64_t)m * d + e];
            dctx[(int64_t)p * d + e] = acc;
            dctr[(int64_t)p * d + e] = g0 * C[(int64_t)p * d + e];
        }
    }
    for (int m = 0; m < M; ++m)
        for (int e = 0; e < d; ++e) {
            double acc = 0.0;
            for (int p = 0; p < P; ++p) acc += G[(int64_t)p * M + m] * C[(int64_t)p * d + e];
            dneg[(int64_t)m * d + e] = acc;
        }
    free(C); free(O); free(N); free(G);
    return loss;
}
