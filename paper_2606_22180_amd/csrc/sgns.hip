// Skip-gram with negative sampling (Train of Algorithm 1; Eq. (1)-(2)).
//
// One minibatch = P consecutive pairs of a chunk's pair order (centre
// position j, then offset slot, then walk).  The pair order is implicit:
// pair g of a chunk is walk valid_cols[g mod Wv] at slice g / Wv, where the
// slice table lists the (j, slot) combinations with both positions inside a
// walk.  Every walk in a chunk has either L nodes or one (an isolated start),
// and the one-node walks are left out of valid_cols, so this closed form is
// exactly the order "next P pairs whose positions both hold a node".
//
// Every pair reads the tables as they stand at the minibatch's start; each
// row's deltas are summed and added once.  FP32 atomics on table rows are
// slow on this part (an L2 atomic unit handles a few dwords per clock, and
// hot rows serialise), so the update is a sort by destination instead:
//   forward   per pair: gather in[ctx], out[ctr], out[neg_1..K]; K+1 dots,
//             sigma, coefficients g; store g and sum_k g_k out[t_k] per pair;
//             count each touched row with an integer atomic whose result is
//             the touch's rank within its row (rank 0 lists the row).
//   scan      two passes over the touched rows: segment offsets and work
//             items (chunks of at most kChunk touches per row).
//   fill      each touch writes its id at its row's offset + rank.
//   reduce    one wave per chunk: out rows sum g * in[ctx] over their
//             touches, in rows sum the per-pair deltas; plain read-modify-
//             write of the row (atomic only for rows split over chunks),
//             and the row's counter is cleared.  Out rows run first, since
//             they read the in-table as of the minibatch start.
// Lanes own elements lane + 64 v of a row, so each row access is one
// coalesced 256-byte transaction per v.
#include <algorithm>

#include "common.h"
#include "noise.h"

namespace felog {

constexpr int kChunk = 16;                 // touches per reduction work item (one per lane of a group)
constexpr uint32_t kFirstChunk = 1u << 31; // flags in chunk_len
constexpr uint32_t kMultiChunk = 1u << 30;
constexpr uint32_t kLenMask = (1u << 30) - 1;

struct SgnsArgs {
    const float* __restrict__ tin;
    const float* __restrict__ tout;
    const int32_t* __restrict__ walks;   // step-major [L][W]
    int64_t W;
    const int32_t* __restrict__ vcols;   // valid columns of this chunk
    uint32_t Wv;
    const int32_t* __restrict__ slices;  // (j << 8) | slot
    uint32_t first_pair;
    uint32_t npairs;
    int64_t id_base;
    int32_t window;
    int32_t ppw;                          // pairs per wave (<= 64 / (K + 2))
    uint64_t seed;
    NoiseTable noise;
    float lr;
    uint32_t* cnt_in;
    uint32_t* cnt_out;
    int32_t* pair_ctx;
    int32_t* pair_t;
    float* pair_g;
    uint32_t* rank_in;
    uint32_t* rank_out;
    float* dinp;
    double* loss_part;                    // one slot per wave
};

// Sum of 8 per-lane values over the wave with 10 exchanges: three halving
// steps leave value k summed over 8-lane groups in lanes 8k..8k+7, then three
// xor steps finish each group.  Returns the total of value k in every lane
// of group k.
__device__ __forceinline__ float reduce8(float v[8], int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        bool hi = lane & 32;
        float send = hi ? v[i] : v[i + 4];
        float keep = hi ? v[i + 4] : v[i];
        v[i] = keep + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        bool hi = lane & 16;
        float send = hi ? v[i] : v[i + 2];
        float keep = hi ? v[i + 2] : v[i];
        v[i] = keep + __shfl_xor(send, 16);
    }
    {
        bool hi = lane & 8;
        float send = hi ? v[0] : v[1];
        float keep = hi ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 8);
    }
    float x = v[0];
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 1);
    return x;   // lane group g = lane >> 3 holds value g
}

__device__ __forceinline__ double wave_sum_f64(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

// -log sigma(x) = log(1 + exp(-x)), evaluated without overflow.
__device__ __forceinline__ double neg_log_sigmoid(double x)
{
    return fmax(-x, 0.0) + log1p(exp(-fabs(x)));
}

// ----------------------------------------------------------------- forward
// A row is handled by a group of 16 lanes (lane j of a group owns the float4s
// j + 16 i of the row), so one wave works on 4 pairs at a time.
template <int D>
__device__ __forceinline__ const float4* row4(const float* base, int64_t row)
{
    return reinterpret_cast<const float4*>(base + row * D);
}

__device__ __forceinline__ float dot4(float4 a, float4 b, float acc)
{
    acc = fmaf(a.x, b.x, acc);
    acc = fmaf(a.y, b.y, acc);
    acc = fmaf(a.z, b.z, acc);
    return fmaf(a.w, b.w, acc);
}

__device__ __forceinline__ float group16_sum(float x)
{
    x += __shfl_xor(x, 8);
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 1);
    return x;
}

template <int D, int K>
__global__ __launch_bounds__(256) void sgns_forward_kernel(SgnsArgs a)
{
    constexpr int V4 = D / 64;   // float4s per lane
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, gl = lane & 15;
    const uint32_t gwave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t q0 = gwave * (uint32_t)a.ppw;
    if (q0 >= a.npairs) return;
    const int np = (int)min((uint32_t)a.ppw, a.npairs - q0);

    // ---- pair metadata: lane p < np handles pair q0 + p
    int32_t m_ctx = 0, m_ctr = 0, m_js = 0, m_col = 0;
    if (lane < np) {
        uint32_t gq = a.first_pair + q0 + lane;
        uint32_t sidx = gq / a.Wv;
        uint32_t rank = gq - sidx * a.Wv;
        m_js = a.slices[sidx];
        m_col = a.vcols[rank];
        int32_t j = m_js >> 8, s = m_js & 255;
        int32_t off = s < a.window ? s - a.window : s - a.window + 1;
        m_ctx = a.walks[(int64_t)(j + off) * a.W + m_col];
        m_ctr = a.walks[(int64_t)j * a.W + m_col];
    }

    // ---- noise draws: lane l < np*K draws negative l % K of pair l / K
    int32_t m_neg = 0;
    {
        int p = lane / K;
        int k = lane - p * K;
        int32_t col = __shfl(m_col, p < np ? p : 0);
        int32_t js = __shfl(m_js, p < np ? p : 0);
        if (lane < np * K) {
            int64_t wid = a.id_base + col;
            Rand4 r = philox4x32((uint32_t)wid, (uint32_t)(wid >> 32), (uint32_t)js,
                                 kTagNeg | (uint32_t)(k >> 1), a.seed);
            uint32_t lo = (k & 1) ? r.v[2] : r.v[0];
            uint32_t hi = (k & 1) ? r.v[3] : r.v[1];
            m_neg = noise_draw(a.noise, ((uint64_t)hi << 32) | lo);
        }
    }

    // ---- rows, dots, coefficients, per-pair in-row delta: 4 pairs at a time
    double lacc = 0.0;
    for (int base = 0; base < np; base += 4) {
        const int p = base + grp;
        const bool live = p < np;
        const int ps = live ? p : 0;
        const uint32_t q = q0 + ps;
        const int32_t ctx = __shfl(m_ctx, ps);
        int32_t t[K + 1];
        t[0] = __shfl(m_ctr, ps);
#pragma unroll
        for (int k = 0; k < K; ++k) t[k + 1] = __shfl(m_neg, ps * K + k);

        float4 vin[V4];
        float4 vo[K + 1][V4];
        const float4* ri = row4<D>(a.tin, ctx);
#pragma unroll
        for (int i = 0; i < V4; ++i) vin[i] = ri[i * 16 + gl];
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            const float4* ro = row4<D>(a.tout, t[k]);
#pragma unroll
            for (int i = 0; i < V4; ++i) vo[k][i] = ro[i * 16 + gl];
        }
        float dot[K + 1];
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            float acc = 0.0f;
#pragma unroll
            for (int i = 0; i < V4; ++i) acc = dot4(vin[i], vo[k][i], acc);
            dot[k] = group16_sum(acc);
        }
        float g[K + 1];
        g[0] = a.lr * (1.0f - sigmoidf_(dot[0]));
#pragma unroll
        for (int k = 1; k <= K; ++k) g[k] = t[k] != t[0] ? -a.lr * sigmoidf_(dot[k]) : 0.0f;

        // lane j of the group stores g_k and takes loss term k for k = j and
        // k = j + 16 (K + 1 may exceed the 16 lanes of a group)
        float s_lo = 0.0f, s_hi = 0.0f;
        bool v_lo = false, v_hi = false;
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            if ((k & 15) == gl) {
                if (live) a.pair_g[q * (K + 1) + k] = g[k];
                const float sk = k == 0 ? dot[0] : -dot[k];   // -log sigma(sk) is the term
                const bool vk = live && (k == 0 || t[k] != t[0]);
                if (k < 16) {
                    s_lo = sk;
                    v_lo = vk;
                } else {
                    s_hi = sk;
                    v_hi = vk;
                }
            }
        }
        if (v_lo) lacc += neg_log_sigmoid((double)s_lo);
        if (K >= 16 && v_hi) lacc += neg_log_sigmoid((double)s_hi);
        if (live) {
            float4* dp = reinterpret_cast<float4*>(a.dinp + (int64_t)q * D);
#pragma unroll
            for (int i = 0; i < V4; ++i) {
                float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                for (int k = 0; k <= K; ++k) {
                    acc.x = fmaf(g[k], vo[k][i].x, acc.x);
                    acc.y = fmaf(g[k], vo[k][i].y, acc.y);
                    acc.z = fmaf(g[k], vo[k][i].z, acc.z);
                    acc.w = fmaf(g[k], vo[k][i].w, acc.w);
                }
                dp[i * 16 + gl] = acc;
            }
        }
    }

    // ---- touches: lane l < np*(K+2) handles touch r = l % (K+2) of pair l / (K+2):
    //      r = 0 centre, 1..K negatives (out table), K+1 context (in table).  The
    //      count's old value is the touch's rank within its row.
    {
        const int p = lane / (K + 2);
        const int r = lane - p * (K + 2);
        const int ps = p < np ? p : 0;
        int32_t ctr = __shfl(m_ctr, ps);
        int32_t ctx = __shfl(m_ctx, ps);
        int32_t neg = __shfl(m_neg, ps * K + (r >= 1 && r <= K ? r - 1 : 0));
        if (lane < np * (K + 2)) {
            const uint32_t q = q0 + p;
            if (r == 0) {
                a.rank_out[q * (K + 1)] = atomicAdd(&a.cnt_out[ctr], 1u);
                a.pair_t[q * (K + 1)] = ctr;
            } else if (r <= K) {
                const bool keep = neg != ctr;
                a.rank_out[q * (K + 1) + r] = keep ? atomicAdd(&a.cnt_out[neg], 1u) : 0u;
                a.pair_t[q * (K + 1) + r] = keep ? neg : -1;
            } else {
                a.rank_in[q] = atomicAdd(&a.cnt_in[ctx], 1u);
                a.pair_ctx[q] = ctx;
            }
        }
    }

    // ---- loss: -log sigma(s0) - sum_k log sigma(-s_k) = softplus(-s0) + sum_k softplus(s_k)
    lacc = wave_sum_f64(lacc);
    if (lane == 0) a.loss_part[gwave] += lacc;
}

// ------------------------------------------------------------------ scan
// Touched rows are the touches of rank 0, listed in touch order: for the in
// table the touches are the pairs (p = 0..P-1), for the out table the
// (pair, slot) ids e = p (K+1) + k.  Scan blocks [0, nb_in) cover the in
// table, the rest the out table; per item the scanned values are
// (rank 0 ? 1 : 0) and (rank 0 ? c : 0 | chunks << 32), c = the row's count.
constexpr int kScanT = 256, kScanI = 8, kScanSpanS = kScanT * kScanI;

struct TouchView {
    const int32_t* pair_ctx;
    const int32_t* pair_t;
    const uint32_t* rank_in;
    const uint32_t* rank_out;
    const uint32_t* cnt_in;
    const uint32_t* cnt_out;
    // row of item i (-1 = not a first touch) and its count
    __device__ void item(bool out, uint32_t i, int32_t& row, uint32_t& c) const
    {
        int32_t r;
        uint32_t rk;
        if (out) {
            r = pair_t[i];
            rk = r >= 0 ? rank_out[i] : 1u;
        } else {
            r = pair_ctx[i];
            rk = rank_in[i];
        }
        row = rk == 0 ? r : -1;
        c = rk == 0 ? (out ? cnt_out[r] : cnt_in[r]) : 0u;
    }
};

__device__ __forceinline__ unsigned long long pack_ec(uint32_t c)
{
    return (unsigned long long)c | ((unsigned long long)((c + kChunk - 1) / kChunk) << 32);
}

__global__ __launch_bounds__(256) void sgns_scan_partials(TouchView tv, uint32_t n_in,
                                                          uint32_t n_out, uint32_t nb_in,
                                                          unsigned long long* part_ec,
                                                          uint32_t* part_rows)
{
    __shared__ unsigned long long lds[kScanT];
    __shared__ uint32_t lds_r[kScanT];
    const bool out = blockIdx.x >= nb_in;
    const uint32_t nb = out ? blockIdx.x - nb_in : blockIdx.x;
    const uint32_t n = out ? n_out : n_in;
    const uint32_t base = nb * kScanSpanS + threadIdx.x * kScanI;
    unsigned long long acc = 0;
    uint32_t rows = 0;
#pragma unroll
    for (int k = 0; k < kScanI; ++k) {
        if (base + k < n) {
            int32_t row;
            uint32_t c;
            tv.item(out, base + k, row, c);
            if (row >= 0) {
                acc += pack_ec(c);
                ++rows;
            }
        }
    }
    lds[threadIdx.x] = acc;
    lds_r[threadIdx.x] = rows;
    __syncthreads();
    for (int s = kScanT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            lds[threadIdx.x] += lds[threadIdx.x + s];
            lds_r[threadIdx.x] += lds_r[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_ec[blockIdx.x] = lds[0];
        part_rows[blockIdx.x] = lds_r[0];
    }
}

struct ScanOut {
    int32_t* list;      // touched rows
    int32_t* off;       // [n] first entry of each row's segment
    int32_t* chunks;    // 4 ints per chunk
};

// meta[0 + out] = rows listed, meta[2 + out] = chunks.
__global__ __launch_bounds__(256) void sgns_scan_write(TouchView tv, uint32_t n_in, uint32_t n_out,
                                                       uint32_t nb_in,
                                                       const unsigned long long* part_ec,
                                                       const uint32_t* part_rows, ScanOut so_in,
                                                       ScanOut so_out, uint32_t* meta)
{
    __shared__ unsigned long long lds[kScanT];
    __shared__ uint32_t lds_r[kScanT];
    const bool out = blockIdx.x >= nb_in;
    const uint32_t b0 = out ? nb_in : 0u;          // first block of this table
    const uint32_t n = out ? n_out : n_in;
    const uint32_t nb = blockIdx.x - b0;
    const ScanOut so = out ? so_out : so_in;
    // offset of this block: partials of the earlier blocks of the same table
    unsigned long long pre = 0;
    uint32_t pre_r = 0;
    for (uint32_t b = b0 + threadIdx.x; b < blockIdx.x; b += kScanT) {
        pre += part_ec[b];
        pre_r += part_rows[b];
    }
    lds[threadIdx.x] = pre;
    lds_r[threadIdx.x] = pre_r;
    __syncthreads();
    for (int s = kScanT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            lds[threadIdx.x] += lds[threadIdx.x + s];
            lds_r[threadIdx.x] += lds_r[threadIdx.x + s];
        }
        __syncthreads();
    }
    const unsigned long long block_ec = lds[0];
    const uint32_t block_r = lds_r[0];
    __syncthreads();

    const uint32_t base = nb * kScanSpanS + threadIdx.x * kScanI;
    int32_t rows[kScanI];
    uint32_t cs[kScanI];
    unsigned long long mine = 0;
    uint32_t mine_r = 0;
#pragma unroll
    for (int k = 0; k < kScanI; ++k) {
        rows[k] = -1;
        cs[k] = 0;
        if (base + k < n) tv.item(out, base + k, rows[k], cs[k]);
        if (rows[k] >= 0) {
            mine += pack_ec(cs[k]);
            ++mine_r;
        }
    }
    // block exclusive scans
    lds[threadIdx.x] = mine;
    lds_r[threadIdx.x] = mine_r;
    __syncthreads();
    for (int off = 1; off < kScanT; off <<= 1) {
        unsigned long long add = threadIdx.x >= off ? lds[threadIdx.x - off] : 0ull;
        uint32_t add_r = threadIdx.x >= off ? lds_r[threadIdx.x - off] : 0u;
        __syncthreads();
        lds[threadIdx.x] += add;
        lds_r[threadIdx.x] += add_r;
        __syncthreads();
    }
    unsigned long long run = block_ec + lds[threadIdx.x] - mine;
    uint32_t slot = block_r + lds_r[threadIdx.x] - mine_r;
    uint32_t entry = (uint32_t)run, chunk = (uint32_t)(run >> 32);
#pragma unroll
    for (int k = 0; k < kScanI; ++k) {
        const uint32_t i = base + k;
        if (rows[k] >= 0) {
            so.list[slot] = rows[k];
            so.off[rows[k]] = (int32_t)entry;
            const uint32_t nch = (cs[k] + kChunk - 1) / kChunk;
            for (uint32_t j = 0; j < nch; ++j) {
                const uint32_t len = min((uint32_t)kChunk, cs[k] - j * kChunk);
                int32_t* d = so.chunks + 4 * (int64_t)(chunk + j);
                d[0] = rows[k];
                d[1] = (int32_t)slot;
                d[2] = (int32_t)(entry + j * kChunk);
                d[3] = (int32_t)(len | (j == 0 ? kFirstChunk : 0u) | (nch > 1 ? kMultiChunk : 0u));
            }
            entry += cs[k];
            chunk += nch;
            ++slot;
        }
        if (i + 1 == n) {       // last item of the table: totals
            meta[out ? 1 : 0] = slot;
            meta[out ? 3 : 2] = chunk;
        }
    }
}

// ------------------------------------------------------------------ fill
template <int K>
__global__ __launch_bounds__(256) void sgns_fill_kernel(uint32_t npairs, const int32_t* pair_ctx,
                                                        const int32_t* pair_t,
                                                        const uint32_t* rank_in,
                                                        const uint32_t* rank_out,
                                                        const int32_t* off_in,
                                                        const int32_t* off_out,
                                                        int32_t* entries_in, int32_t* entries_out)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < npairs * (K + 1)) {
        const int32_t row = pair_t[t];
        if (row >= 0) entries_out[off_out[row] + rank_out[t]] = (int32_t)t;
    } else if (t < npairs * (K + 2)) {
        const uint32_t p = t - npairs * (K + 1);
        entries_in[off_in[pair_ctx[p]] + rank_in[p]] = (int32_t)p;
    }
}

// ---------------------------------------------------------------- reduce
// Out rows: delta out[t] = sum over touches (p, k) of g_pk * in[ctx_p].
// In rows:  delta in[c]  = sum over touches p of dinp[p].
// Groups of 16 lanes take one chunk each, 4 chunks per wave.  capture !=
// NULL: write the deltas to capture[slot][d] (zeroed) instead of the table.
template <int D, int K, bool OUT>
__global__ __launch_bounds__(256) void sgns_reduce_kernel(
    float* __restrict__ table, const float* __restrict__ tin, const float* __restrict__ dinp,
    const float* __restrict__ pair_g, const int32_t* __restrict__ pair_ctx,
    const int32_t* __restrict__ entries, const int32_t* __restrict__ chunks,
    uint32_t* __restrict__ cnt, const uint32_t* meta, float* __restrict__ capture,
    unsigned long long* row_totals)
{
    constexpr int V4 = D / 64;
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, gl = lane & 15;
    const uint32_t n_chunks = meta[OUT ? 3 : 2];
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    const float* src = OUT ? tin : dinp;
    for (uint32_t base = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 4u;
         base < n_chunks; base += nw * 4u) {
        const uint32_t c = base + grp;
        const bool live = c < n_chunks;
        int32_t row = 0, slot = 0, start = 0, len = 0;
        uint32_t lf = 0;
        if (live) {
            const int4 d = reinterpret_cast<const int4*>(chunks)[c];
            row = d.x;
            slot = d.y;
            start = d.z;
            lf = (uint32_t)d.w;
            len = (int32_t)(lf & kLenMask);
        }
        float my_g = 0.0f;
        int32_t my_src = 0;
        if (gl < len) {
            const int32_t e = entries[start + gl];
            if (OUT) {
                my_g = pair_g[e];
                my_src = pair_ctx[e / (K + 1)];
            } else {
                my_g = 1.0f;
                my_src = e;
            }
        }
        // longest chunk among the wave's four groups
        int32_t mlen = max(len, __shfl_xor(len, 16));
        mlen = max(mlen, __shfl_xor(mlen, 32));
        float4 acc[V4];
#pragma unroll
        for (int i = 0; i < V4; ++i) acc[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int32_t i0 = 0; i0 < mlen; i0 += 4) {
            float gg[4];
            float4 x[4][V4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t idx = min(i0 + u, kChunk - 1);
                gg[u] = __shfl(my_g, (grp << 4) + idx);
                const int32_t rr = __shfl(my_src, (grp << 4) + idx);
                if (i0 + u < len) {
                    const float4* rp = row4<D>(src, rr);
#pragma unroll
                    for (int i = 0; i < V4; ++i) x[u][i] = rp[i * 16 + gl];
                } else {
                    gg[u] = 0.0f;
#pragma unroll
                    for (int i = 0; i < V4; ++i) x[u][i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int i = 0; i < V4; ++i) {
                    acc[i].x = fmaf(gg[u], x[u][i].x, acc[i].x);
                    acc[i].y = fmaf(gg[u], x[u][i].y, acc[i].y);
                    acc[i].z = fmaf(gg[u], x[u][i].z, acc[i].z);
                    acc[i].w = fmaf(gg[u], x[u][i].w, acc[i].w);
                }
        }
        if (live) {
            float* dst = capture ? capture + (int64_t)slot * D : table + (int64_t)row * D;
            float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
            for (int i = 0; i < V4; ++i) {
                if (lf & kMultiChunk) {
                    float* f = dst + (i * 16 + gl) * 4;
                    unsafeAtomicAdd(f + 0, acc[i].x);
                    unsafeAtomicAdd(f + 1, acc[i].y);
                    unsafeAtomicAdd(f + 2, acc[i].z);
                    unsafeAtomicAdd(f + 3, acc[i].w);
                } else if (capture) {
                    d4[i * 16 + gl] = acc[i];
                } else {
                    float4 v = d4[i * 16 + gl];
                    v.x += acc[i].x;
                    v.y += acc[i].y;
                    v.z += acc[i].z;
                    v.w += acc[i].w;
                    d4[i * 16 + gl] = v;
                }
            }
            if ((lf & kFirstChunk) && gl == 0) cnt[row] = 0;
        }
    }
    // the in-row reduction is the minibatch's last kernel: count the touched rows
    if (!OUT && blockIdx.x == 0 && threadIdx.x == 0) {
        row_totals[0] += meta[0];
        row_totals[1] += meta[1];
    }
}

// Fixed-order FP64 sum of the per-wave loss partials (one block).
__global__ __launch_bounds__(256) void loss_reduce_kernel(const double* part, int64_t n,
                                                          double* out)
{
    __shared__ double lds[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[i];
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = lds[0];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// (j, slot) slices with both positions inside a walk of length L, in pair order.
static std::vector<int32_t> make_slices(int32_t L, int32_t w)
{
    std::vector<int32_t> out;
    for (int32_t j = 0; j < L; ++j)
        for (int32_t s = 0; s < 2 * w; ++s) {
            int32_t off = s < w ? s - w : s - w + 1;
            if (j + off >= 0 && j + off < L) out.push_back((j << 8) | s);
        }
    return out;
}

static TrainSchedule make_schedule(Walks& w, const felog_train_params& p)
{
    int64_t chunk = p.chunk_walks ? p.chunk_walks : (int64_t)1 << 20;
    launch_valid_columns(w, chunk);
    TrainSchedule s;
    s.nslices = (int64_t)make_slices(w.L, p.window).size();
    int64_t base = 0;
    for (size_t c = 0; c < w.chunk_valid.size(); ++c) {
        int64_t pairs = w.chunk_valid[c] * s.nslices;
        FELOG_REQUIRE(pairs < ((int64_t)1 << 32),
                      "a chunk yields %lld pairs; at most 2^32 - 1 are supported (use a "
                      "smaller chunk_walks)", (long long)pairs);
        s.chunk_first_mb.push_back(s.B);
        s.chunk_pairs.push_back(pairs);
        s.chunk_valid_base.push_back(base);
        base += w.chunk_valid[c];
        s.B += (pairs + p.minibatch_pairs - 1) / p.minibatch_pairs;
        s.total_pairs += pairs;
    }
    return s;
}

int64_t count_minibatches(Walks& w, const felog_train_params& p, int64_t* total_pairs)
{
    TrainSchedule s = make_schedule(w, p);
    if (total_pairs) *total_pairs = s.total_pairs;
    return s.B;
}


struct MinibatchLaunch {
    dim3 fwd_grid;
    uint32_t npairs;
    int dim, K;
    int fill_blocks, reduce_blocks;
    uint32_t nb_in, nb_out;
};

template <int D, int K>
static void launch_minibatch_t(Model& m, const SgnsArgs& a, const MinibatchLaunch& ml,
                               float* cap_in, float* cap_out, hipStream_t s, hipEvent_t ev_mid)
{
    hipLaunchKernelGGL((sgns_forward_kernel<D, K>), ml.fwd_grid, dim3(256), 0, s, a);
    if (ev_mid) FELOG_HIP(hipEventRecord(ev_mid, s));
    TouchView tv{m.pair_ctx.as<int32_t>(), m.pair_t.as<int32_t>(), m.rank_in.as<uint32_t>(),
                 m.rank_out.as<uint32_t>(), m.cnt_in.as<uint32_t>(), m.cnt_out.as<uint32_t>()};
    uint32_t* meta = m.meta.as<uint32_t>();
    const uint32_t n_in = ml.npairs, n_out = ml.npairs * (K + 1);
    const uint32_t nb = ml.nb_in + ml.nb_out;
    unsigned long long* part_ec = m.partials.as<unsigned long long>();
    uint32_t* part_rows = reinterpret_cast<uint32_t*>(part_ec + nb);
    hipLaunchKernelGGL(sgns_scan_partials, dim3(nb), dim3(256), 0, s, tv, n_in, n_out, ml.nb_in,
                       part_ec, part_rows);
    ScanOut so_in{m.list_in.as<int32_t>(), m.off_in.as<int32_t>(), m.chunks_in.as<int32_t>()};
    ScanOut so_out{m.list_out.as<int32_t>(), m.off_out.as<int32_t>(), m.chunks_out.as<int32_t>()};
    hipLaunchKernelGGL(sgns_scan_write, dim3(nb), dim3(256), 0, s, tv, n_in, n_out, ml.nb_in,
                       part_ec, part_rows, so_in, so_out, meta);
    hipLaunchKernelGGL(sgns_fill_kernel<K>, dim3(ml.fill_blocks), dim3(256), 0, s, ml.npairs,
                       m.pair_ctx.as<int32_t>(), m.pair_t.as<int32_t>(),
                       m.rank_in.as<uint32_t>(), m.rank_out.as<uint32_t>(),
                       m.off_in.as<int32_t>(), m.off_out.as<int32_t>(),
                       m.entries_in.as<int32_t>(), m.entries_out.as<int32_t>());
    hipLaunchKernelGGL((sgns_reduce_kernel<D, K, true>), dim3(ml.reduce_blocks), dim3(256), 0, s,
                       m.tout.as<float>(), m.tin.as<float>(), m.dinp.as<float>(),
                       m.pair_g.as<float>(), m.pair_ctx.as<int32_t>(), m.entries_out.as<int32_t>(),
                       m.chunks_out.as<int32_t>(), m.cnt_out.as<uint32_t>(), meta, cap_out,
                       m.row_totals.as<unsigned long long>());
    hipLaunchKernelGGL((sgns_reduce_kernel<D, K, false>), dim3(ml.reduce_blocks), dim3(256), 0, s,
                       m.tin.as<float>(), m.tin.as<float>(), m.dinp.as<float>(),
                       m.pair_g.as<float>(), m.pair_ctx.as<int32_t>(), m.entries_in.as<int32_t>(),
                       m.chunks_in.as<int32_t>(), m.cnt_in.as<uint32_t>(), meta, cap_in,
                       m.row_totals.as<unsigned long long>());
    FELOG_HIP(hipGetLastError());
}

template <int D>
static void launch_minibatch_k(int K, Model& m, const SgnsArgs& a, const MinibatchLaunch& ml,
                               float* ci, float* co, hipStream_t s, hipEvent_t ev)
{
    switch (K) {
#define FELOG_K(k) case k: launch_minibatch_t<D, k>(m, a, ml, ci, co, s, ev); break;
        FELOG_K(1) FELOG_K(2) FELOG_K(3) FELOG_K(4) FELOG_K(5) FELOG_K(6) FELOG_K(7)
        FELOG_K(8) FELOG_K(9) FELOG_K(10) FELOG_K(11) FELOG_K(12) FELOG_K(13) FELOG_K(14)
        FELOG_K(15) FELOG_K(16) FELOG_K(17) FELOG_K(18) FELOG_K(19) FELOG_K(20)
#undef FELOG_K
        default: fail(FELOG_EUNSUPPORTED, "negatives = %d not supported", K);
    }
}

static void launch_minibatch(Model& m, const SgnsArgs& a, const MinibatchLaunch& ml, float* ci,
                             float* co, hipStream_t s, hipEvent_t ev)
{
    if (ml.dim == 64) launch_minibatch_k<64>(ml.K, m, a, ml, ci, co, s, ev);
    else if (ml.dim == 128) launch_minibatch_k<128>(ml.K, m, a, ml, ci, co, s, ev);
    else launch_minibatch_k<256>(ml.K, m, a, ml, ci, co, s, ev);
}

void train_minibatches(Model& m, const Walks& wc, const felog_train_params& p, int64_t first_mb,
                       int64_t n_mb, bool apply, felog_train_stats* stats, int32_t* rows_in,
                       float* d_in_host, int64_t cap_in, int64_t* n_in, int32_t* rows_out,
                       float* d_out_host, int64_t cap_out, int64_t* n_out)
{
    Walks& w = const_cast<Walks&>(wc);
    Ctx& c = *m.ctx;
    c.make_current();
    TrainSchedule sch = make_schedule(w, p);
    const int K = p.negatives;
    const int64_t P = p.minibatch_pairs;
    int64_t end = n_mb < 0 ? sch.B : std::min<int64_t>(sch.B, first_mb + n_mb);
    if (first_mb > sch.B) first_mb = sch.B;
    if (!apply) FELOG_REQUIRE(first_mb < sch.B, "minibatch %lld out of range (%lld minibatches)",
                              (long long)first_mb, (long long)sch.B);

    if (m.precision == FELOG_PREC_BF16) {
        std::vector<int32_t> sl = make_slices(w.L, p.window);
        DevBuf slices;
        slices.alloc(&c, sizeof(int32_t) * std::max<size_t>(sl.size(), 1));
        if (!sl.empty())
            FELOG_HIP(hipMemcpyAsync(slices.ptr, sl.data(), sizeof(int32_t) * sl.size(),
                                     hipMemcpyHostToDevice, c.stream));
        if (apply) {
            train_minibatches_bf16(m, w, p, sch, slices.as<int32_t>(), first_mb, end, nullptr,
                                   nullptr, stats);
            return;
        }
        // capture: deltas into dense zeroed tables, then the touched rows
        const int64_t cnt = (int64_t)m.g->n * m.dim;
        FELOG_REQUIRE(cnt <= ((int64_t)1 << 28), "delta capture of a BF16 model is limited to "
                      "n * d <= 2^28");
        DevBuf din, dout;
        din.alloc(&c, sizeof(float) * cnt);
        dout.alloc(&c, sizeof(float) * cnt);
        FELOG_HIP(hipMemsetAsync(din.ptr, 0, din.bytes, c.stream));
        FELOG_HIP(hipMemsetAsync(dout.ptr, 0, dout.bytes, c.stream));
        felog_train_stats st{};
        train_minibatches_bf16(m, w, p, sch, slices.as<int32_t>(), first_mb, first_mb + 1,
                               din.as<float>(), dout.as<float>(), &st);
        std::vector<int32_t> ids(2 * (size_t)p.minibatch_pairs + p.shared_negatives);
        FELOG_HIP(hipMemcpyAsync(ids.data(), m.bf_ids.ptr, sizeof(int32_t) * ids.size(),
                                 hipMemcpyDeviceToHost, c.stream));
        std::vector<float> hin(cnt), hout(cnt);
        FELOG_HIP(hipMemcpyAsync(hin.data(), din.ptr, sizeof(float) * cnt, hipMemcpyDeviceToHost,
                                 c.stream));
        FELOG_HIP(hipMemcpyAsync(hout.data(), dout.ptr, sizeof(float) * cnt,
                                 hipMemcpyDeviceToHost, c.stream));
        c.sync();
        std::vector<char> seen_in(m.g->n, 0), seen_out(m.g->n, 0);
        int64_t ui = 0, uo = 0;
        const int64_t Pn = p.minibatch_pairs;
        auto put = [&](int32_t row, bool out) {
            std::vector<char>& seen = out ? seen_out : seen_in;
            if (row < 0 || seen[row]) return;
            seen[row] = 1;
            int64_t& u = out ? uo : ui;
            FELOG_REQUIRE(u < (out ? cap_out : cap_in), "capture buffers too small");
            (out ? rows_out : rows_in)[u] = row;
            std::copy_n((out ? hout : hin).data() + (int64_t)row * m.dim, m.dim,
                        (out ? d_out_host : d_in_host) + u * m.dim);
            ++u;
        };
        for (int64_t q = 0; q < Pn; ++q) put(ids[q], false);
        for (int64_t q = 0; q < Pn; ++q) if (ids[q] >= 0) put(ids[Pn + q], true);
        for (int64_t q = 0; q < p.shared_negatives; ++q) put(ids[2 * Pn + q], true);
        if (n_in) *n_in = ui;
        if (n_out) *n_out = uo;
        if (stats) *stats = st;
        return;
    }

    // scratch sized for this minibatch size
    if (m.cap_pairs < P || m.cap_K < K) {
        m.cap_pairs = std::max<int64_t>(m.cap_pairs, P);
        m.cap_K = std::max(m.cap_K, K);
        const int64_t cp = m.cap_pairs, ck = m.cap_K;
        m.pair_ctx.alloc(&c, sizeof(int32_t) * cp);
        m.pair_t.alloc(&c, sizeof(int32_t) * cp * (ck + 1));
        m.pair_g.alloc(&c, sizeof(float) * cp * (ck + 1));
        m.rank_in.alloc(&c, sizeof(uint32_t) * cp);
        m.rank_out.alloc(&c, sizeof(uint32_t) * cp * (ck + 1));
        m.dinp.alloc(&c, sizeof(float) * cp * m.dim);
        m.list_in.alloc(&c, sizeof(int32_t) * cp);
        m.list_out.alloc(&c, sizeof(int32_t) * cp * (ck + 1));
        m.entries_in.alloc(&c, sizeof(int32_t) * cp);
        m.entries_out.alloc(&c, sizeof(int32_t) * cp * (ck + 1));
        m.chunks_in.alloc(&c, sizeof(int32_t) * 4 * cp);
        m.chunks_out.alloc(&c, sizeof(int32_t) * 4 * cp * (ck + 1));
        const int64_t nbmax = (cp + kScanSpanS - 1) / kScanSpanS +
                              (cp * (ck + 1) + kScanSpanS - 1) / kScanSpanS;
        m.partials.alloc(&c, (sizeof(unsigned long long) + sizeof(uint32_t)) * nbmax);
    }
    const int ppw_max = 64 / (K + 2);
    int ppw = (int)std::min<int64_t>(ppw_max, std::max<int64_t>(1, P / ((int64_t)c.num_cus * 32)));
    const int64_t waves = (P + ppw - 1) / ppw;
    const int64_t blocks = (waves + 3) / 4;
    DevBuf loss_part;
    loss_part.alloc(&c, sizeof(double) * blocks * 4);
    FELOG_HIP(hipMemsetAsync(loss_part.ptr, 0, sizeof(double) * blocks * 4, c.stream));
    FELOG_HIP(hipMemsetAsync(m.meta.ptr, 0, sizeof(uint32_t) * 8, c.stream));
    FELOG_HIP(hipMemsetAsync(m.row_totals.ptr, 0, sizeof(uint64_t) * 2, c.stream));

    // sampled kernel timing: events before forward, after forward, after the reductions
    const int every = apply ? c.timing_every : 0;
    const size_t pool = c.timing_pool.size() / 3;
    size_t next_slot = 0, used_slots = 0;
    int64_t timed = 0;
    double ms_fwd = 0.0, ms_apply = 0.0;
    auto harvest = [&](size_t slot) {
        hipEvent_t* e = &c.timing_pool[3 * slot];
        FELOG_HIP(hipEventSynchronize(e[2]));
        float f = 0.0f, ap = 0.0f;
        FELOG_HIP(hipEventElapsedTime(&f, e[0], e[1]));
        FELOG_HIP(hipEventElapsedTime(&ap, e[1], e[2]));
        ms_fwd += f;
        ms_apply += ap;
        ++timed;
    };

    std::vector<int32_t> sl = make_slices(w.L, p.window);
    DevBuf slices;
    slices.alloc(&c, sizeof(int32_t) * std::max<size_t>(sl.size(), 1));
    if (!sl.empty())
        FELOG_HIP(hipMemcpyAsync(slices.ptr, sl.data(), sizeof(int32_t) * sl.size(),
                                 hipMemcpyHostToDevice, c.stream));

    SgnsArgs a{};
    a.tin = m.tin.as<float>();
    a.tout = m.tout.as<float>();
    a.walks = w.data.as<int32_t>();
    a.W = w.W;
    a.slices = slices.as<int32_t>();
    a.id_base = w.id_base;
    a.window = p.window;
    a.ppw = ppw;
    a.seed = p.seed;
    a.noise = NoiseTable{m.cdf.as<uint64_t>(), m.guide.as<int32_t>(), m.total_weight, m.guide_bits};
    a.cnt_in = m.cnt_in.as<uint32_t>();
    a.cnt_out = m.cnt_out.as<uint32_t>();
    a.pair_ctx = m.pair_ctx.as<int32_t>();
    a.pair_t = m.pair_t.as<int32_t>();
    a.pair_g = m.pair_g.as<float>();
    a.rank_in = m.rank_in.as<uint32_t>();
    a.rank_out = m.rank_out.as<uint32_t>();
    a.dinp = m.dinp.as<float>();
    a.loss_part = loss_part.as<double>();

    MinibatchLaunch ml{};
    ml.dim = m.dim;
    ml.K = K;
    ml.reduce_blocks = std::max(1, c.num_cus * 8);

    const double lr0 = (double)p.lr_start, lr1 = (double)p.lr_end;
    int64_t pairs_done = 0;
    FELOG_HIP(hipEventRecord(c.ev0, c.stream));
    size_t chunk = 0;
    for (int64_t b = first_mb; b < end; ++b) {
        while (chunk + 1 < sch.chunk_first_mb.size() && sch.chunk_first_mb[chunk + 1] <= b) ++chunk;
        int64_t local = b - sch.chunk_first_mb[chunk];
        int64_t first = local * P;
        int64_t np = std::min<int64_t>(P, sch.chunk_pairs[chunk] - first);
        a.vcols = w.valid_cols.as<int32_t>() + sch.chunk_valid_base[chunk];
        a.Wv = (uint32_t)w.chunk_valid[chunk];
        a.first_pair = (uint32_t)first;
        a.npairs = (uint32_t)np;
        double lr = lr0 - (lr0 - lr1) * (double)b / (double)std::max<int64_t>(1, sch.B - 1);
        a.lr = (float)lr;
        int64_t nwaves = (np + ppw - 1) / ppw;
        ml.fwd_grid = dim3((uint32_t)((nwaves + 3) / 4));
        ml.npairs = (uint32_t)np;
        ml.fill_blocks = (int)((np * (K + 2) + 255) / 256);
        ml.nb_in = (uint32_t)((np + kScanSpanS - 1) / kScanSpanS);
        ml.nb_out = (uint32_t)((np * (K + 1) + kScanSpanS - 1) / kScanSpanS);
        const bool timed_mb = every > 0 && pool > 0 && (b - first_mb) % every == 0;
        hipEvent_t* ev = nullptr;
        if (timed_mb) {
            if (used_slots == pool) harvest(next_slot);   // reuse the oldest slot
            else ++used_slots;
            ev = &c.timing_pool[3 * next_slot];
            next_slot = (next_slot + 1) % pool;
            FELOG_HIP(hipEventRecord(ev[0], c.stream));
        }
        if (apply) {
            launch_minibatch(m, a, ml, nullptr, nullptr, c.stream, ev ? ev[1] : nullptr);
            if (ev) FELOG_HIP(hipEventRecord(ev[2], c.stream));
        } else {
            // capture: deltas of this minibatch, by touched-list position, not applied
            DevBuf vin, vout;
            vin.alloc(&c, sizeof(float) * (size_t)P * m.dim);
            vout.alloc(&c, sizeof(float) * (size_t)P * (K + 1) * m.dim);
            FELOG_HIP(hipMemsetAsync(vin.ptr, 0, vin.bytes, c.stream));
            FELOG_HIP(hipMemsetAsync(vout.ptr, 0, vout.bytes, c.stream));
            // the last kernel adds the list lengths to row_totals (zeroed above)
            FELOG_HIP(hipMemsetAsync(m.row_totals.ptr, 0, sizeof(uint64_t) * 2, c.stream));
            launch_minibatch(m, a, ml, vin.as<float>(), vout.as<float>(), c.stream, nullptr);
            unsigned long long tot[2];
            FELOG_HIP(hipMemcpyAsync(tot, m.row_totals.ptr, sizeof tot, hipMemcpyDeviceToHost,
                                     c.stream));
            c.sync();
            const int64_t ui = (int64_t)tot[0], uo = (int64_t)tot[1];
            FELOG_REQUIRE(rows_in && d_in_host && rows_out && d_out_host,
                          "capture buffers must not be NULL");
            FELOG_REQUIRE(ui <= cap_in && uo <= cap_out,
                          "capture buffers hold %lld / %lld rows, need %lld / %lld",
                          (long long)cap_in, (long long)cap_out, (long long)ui, (long long)uo);
            FELOG_HIP(hipMemcpyAsync(rows_in, m.list_in.ptr, sizeof(int32_t) * ui,
                                     hipMemcpyDeviceToHost, c.stream));
            FELOG_HIP(hipMemcpyAsync(rows_out, m.list_out.ptr, sizeof(int32_t) * uo,
                                     hipMemcpyDeviceToHost, c.stream));
            FELOG_HIP(hipMemcpyAsync(d_in_host, vin.ptr, sizeof(float) * ui * m.dim,
                                     hipMemcpyDeviceToHost, c.stream));
            FELOG_HIP(hipMemcpyAsync(d_out_host, vout.ptr, sizeof(float) * uo * m.dim,
                                     hipMemcpyDeviceToHost, c.stream));
            FELOG_HIP(hipMemsetAsync(m.row_totals.ptr, 0, sizeof(uint64_t) * 2, c.stream));
            c.sync();
            if (n_in) *n_in = ui;
            if (n_out) *n_out = uo;
        }
        pairs_done += np;
    }
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, c.stream,
                       loss_part.as<double>(), blocks * 4, m.loss_out.as<double>());
    FELOG_HIP(hipGetLastError());
    FELOG_HIP(hipEventRecord(c.ev1, c.stream));
    double loss = 0.0;
    unsigned long long rows[2] = {0, 0};
    FELOG_HIP(hipMemcpyAsync(&loss, m.loss_out.ptr, sizeof loss, hipMemcpyDeviceToHost, c.stream));
    FELOG_HIP(hipMemcpyAsync(rows, m.row_totals.ptr, sizeof rows, hipMemcpyDeviceToHost,
                             c.stream));
    c.sync();
    // harvest the slots still pending, oldest first
    for (size_t k = 0; k < used_slots; ++k)
        harvest((next_slot + pool - used_slots + k) % pool);
    float ms = 0.0f;
    FELOG_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    if (stats) {
        stats->minibatches = end - first_mb;
        stats->pairs = pairs_done;
        stats->minibatches_total = sch.B;
        stats->loss = loss;
        stats->ms = ms;
        stats->rows_in = (int64_t)rows[0];
        stats->rows_out = (int64_t)rows[1];
        stats->timed_launches = timed;
        stats->ms_forward = ms_fwd;
        stats->ms_apply = ms_apply;
    }
}

}  // namespace felog
