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
// row's deltas are summed and added once.  A pair touches K + 2 rows: its
// context (in-table) and its centre and K negatives (out-table).  FP32
// atomics on table rows are slow on this part (an L2 atomic unit handles a
// few dwords per clock and hot rows serialise), so the deltas are sorted by
// destination row instead.  Per minibatch:
//   prep     one thread per touch: node ids (walk reads, noise draws) and an
//            integer atomic per touched row whose old value is the touch's
//            rank within the row (rank 0 marks the row's first touch).
//   scan     two passes over the touches: segment offsets of the touched
//            rows, their list, one work item per row of at most kChunk
//            touches and one per kChunk touches of the rows with more.  No
//            atomics: same-address device atomics serialise at about one per
//            12 ns on this part.
//   forward  one group of 16 lanes (d = 64) or 32 (d >= 128) per pair: gather
//            in[ctx], out[ctr], out[neg_1..K]; K+1 dots, sigma and the
//            coefficients g in FP64 over the FP32 entries; writes (g_k, ctx)
//            and the touch's pair-order key at the out-row's segment
//            position, sum_k g_k out[t_k] (rounded to FP32 once) and the pair
//            at the in-row's; out rows touched once are updated in place.
//   split    chunks of the rows with more than kChunk touches: exact sums
//            (below), stored per chunk.
//   reduce   rows of at most kChunk touches, out rows first (they read the
//            in-table as of the minibatch start), then in rows: the touches
//            are sorted by key inside a 16-lane group and their terms summed
//            in FP64 in pair order, added to the row with one rounding.
//   merge    each split row adds its chunks' sums in chunk order.
// prep and scan read only the walks and the noise table, so with two sets
// of their buffers the next minibatch's run on a second stream while this
// one trains.  Every sum is independent of the order the atomics produced,
// so a minibatch's update is bit-identical from run to run.  The split rows'
// sums are exact: each term (an exact FP64 product g * x, or an FP32 per-pair
// delta) is bounded by lr 2^15 in magnitude and rounded once to a multiple
// of 2^(e - 35), e = floor(log2 lr); in FP64, sums of such multiples below
// lr 2^17 carry no rounding error in any order.
// Lanes own elements 4 (gl + 16 i) .. +3 of a row, so each row access is a
// coalesced 256-byte transaction per i.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "noise.h"
#include "sgns_device.h"

namespace felog {

// ------------------------------------------------------------------- prep
struct PrepArgs {
    const int32_t* __restrict__ walks;   // step-major [L][W]
    int64_t W;
    const int32_t* __restrict__ vcols;   // valid columns of this chunk
    uint32_t Wv;
    const int32_t* __restrict__ slices;  // (j << 8) | slot
    uint32_t first_pair;
    uint32_t npairs;
    int64_t id_base;
    int32_t window;
    uint64_t seed;
    NoiseTable noise;
    uint32_t* cnt_in;
    uint32_t* cnt_out;
    int32_t* touch_row;      // [P][K+2]: context, centre, negatives (-1: negative == centre)
    uint32_t* touch_pos;     // [P][K+2]: rank of the touch within its row
};

// Grid-stride over the touches: the launch is capped at a few blocks per CU,
// which leaves room for the training launches it runs beside.
template <int K>
__global__ __launch_bounds__(256) void sgns_prep_kernel(PrepArgs a)
{
    const uint32_t nt = a.npairs * (K + 2);
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < nt; t += gridDim.x * 256) {
        int32_t row = -1;
        bool out = false;
        const uint32_t p = t / (K + 2), r = t - p * (K + 2);
        const uint32_t gq = a.first_pair + p;
        const uint32_t sidx = gq / a.Wv;
        const uint32_t rank = gq - sidx * a.Wv;
        const int32_t js = a.slices[sidx];
        const int32_t col = a.vcols[rank];
        const int32_t j = js >> 8, s = js & 255;
        const int32_t ctr = a.walks[(int64_t)j * a.W + col];
        if (r == 0) {
            const int32_t off = s < a.window ? s - a.window : s - a.window + 1;
            row = a.walks[(int64_t)(j + off) * a.W + col];
        } else if (r == 1) {
            row = ctr;
            out = true;
        } else {
            // negative k = r - 2: Philox(walk id, (j << 8) | slot, NEG | k / 2), words
            // 2 (k mod 2) and 2 (k mod 2) + 1
            const uint32_t k = r - 2;
            const int64_t wid = a.id_base + col;
            const Rand4 x = philox4x32((uint32_t)wid, (uint32_t)(wid >> 32), (uint32_t)js,
                                       kTagNeg | (k >> 1), a.seed);
            const uint32_t lo = (k & 1) ? x.v[2] : x.v[0];
            const uint32_t hi = (k & 1) ? x.v[3] : x.v[1];
            const int32_t neg = noise_draw(a.noise, ((uint64_t)hi << 32) | lo);
            row = neg != ctr ? neg : -1;   // a negative equal to the centre is skipped
            out = true;
        }
        a.touch_row[t] = row;
        a.touch_pos[t] = row >= 0 ? atomicAdd((out ? a.cnt_out : a.cnt_in) + row, 1u) : 0u;
    }
}

// ------------------------------------------------------------------- scan
// Items: the in-touches i (touch i (K+2)) and, in further blocks, the
// out-touches e (touch (e / (K+1)) (K+2) + 1 + e mod (K+1)).  A first touch
// (rank 0) lists its row; the scanned values are (entries | chunks << 32),
// the rows listed, the rows split over chunks, their chunks and the out rows
// touched once (which the forward updates itself).  A thread takes I items:
// 2 up to 65,536 pairs per minibatch (shorter chains of dependent loads per
// thread and more blocks than with 8; on R-MAT 2^20, d = 128, K = 5:
// 39.5 -> 34.0 us per minibatch at P = 1,024, 73.2 -> 64.7 at 16,384,
// 146.3 -> 142.7 at 65,536), 8 above, where every block's sum over the
// partials of the blocks before it (quadratic in their number) would grow.
constexpr int kScanT = 256;
constexpr int kScanISmall = 2, kScanILarge = 8;
constexpr int64_t kScanSmallPairs = 65536;
static_assert(kScanT * kScanISmall == kScanSpanMin, "fewest items per scan block");

struct ScanArgs {
    const int32_t* touch_row;
    const uint32_t* touch_pos;
    const uint32_t* cnt_in;
    uint32_t* cnt_out;
    uint32_t n_in, n_out, nb_in;
    unsigned long long* part_ec;   // per block
    uint4* part_rm;                // per block: rows, split rows, chunks of split rows,
                                   // single-touch out rows
    int32_t* list_in;
    int32_t* list_out;
    int32_t* off_in;
    int32_t* off_out;
    int4* chunks_in;
    int4* chunks_out;
    int4* split_in;                // chunks of split rows: row, first entry, length, partial row
    int4* split_out;
    int4* mrows_in;                // split rows: row, first chunk, chunks, list slot
    int4* mrows_out;
    uint32_t* meta;
    int32_t reset;                 // zero the counters of the rows done here (else the
                                   // whole counter arrays are zeroed before the ids)
};

// Items base .. base + I - 1 of a table (n items): the row each one
// lists (-1 if none) and the row's touch count.  BATCH issues the loads of
// all the items before it uses any (indices past the end clamped, their
// values dropped): two round trips to memory instead of 2 I, for when
// the scan is on the minibatch's critical path.  Otherwise each item's loads
// wait for the previous item, which leaves more bandwidth to the launches
// that run beside the scan.
template <int K, bool BATCH, int I>
__device__ __forceinline__ void scan_items(const ScanArgs& a, bool out, uint32_t base, uint32_t n,
                                           int32_t (&rows)[I], uint32_t (&cs)[I])
{
    const uint32_t* cnt = out ? a.cnt_out : a.cnt_in;
    if (BATCH) {
        const uint32_t last = n > 0 ? n - 1 : 0;
        uint32_t pos[I];
#pragma unroll
        for (int k = 0; k < I; ++k) {
            const uint32_t i = min(base + k, last);
            const uint32_t t = out ? (i / (K + 1)) * (K + 2) + 1 + i % (K + 1) : i * (K + 2);
            rows[k] = a.touch_row[t];
            pos[k] = a.touch_pos[t];
        }
#pragma unroll
        for (int k = 0; k < I; ++k) {
            const bool first = base + k < n && rows[k] >= 0 && pos[k] == 0u;
            rows[k] = first ? rows[k] : -1;
            cs[k] = cnt[first ? rows[k] : 0];
        }
#pragma unroll
        for (int k = 0; k < I; ++k) cs[k] = rows[k] >= 0 ? cs[k] : 0u;
    } else {
#pragma unroll
        for (int k = 0; k < I; ++k) {
            rows[k] = -1;
            cs[k] = 0u;
            if (base + k < n) {
                const uint32_t i = base + k;
                const uint32_t t = out ? (i / (K + 1)) * (K + 2) + 1 + i % (K + 1) : i * (K + 2);
                const int32_t r = a.touch_row[t];
                if (r >= 0 && a.touch_pos[t] == 0u) {
                    rows[k] = r;
                    cs[k] = cnt[r];
                }
            }
        }
    }
}

__device__ __forceinline__ uint4 add4(uint4 a, uint4 b)
{
    return make_uint4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

// An out row with a single touch in the minibatch is read and written by that
// touch's pair only, so the forward adds its delta in place: it gets no
// segment entry and no work item.
__device__ __forceinline__ bool single_out(uint32_t c, bool out) { return out && c == 1u; }

__device__ __forceinline__ uint4 split_counts(uint32_t c, bool out)
{
    const uint32_t nch = (c + kChunk - 1) / kChunk;
    return make_uint4(1u, nch > 1 ? 1u : 0u, nch > 1 ? nch : 0u, single_out(c, out) ? 1u : 0u);
}

__device__ __forceinline__ unsigned long long pack_ec(uint32_t c, bool out)
{
    const uint32_t e = single_out(c, out) ? 0u : c;
    return (unsigned long long)e | ((unsigned long long)((e + kChunk - 1) / kChunk) << 32);
}

template <int K, bool BATCH, int I>
__global__ __launch_bounds__(256) void sgns_scan_partials(ScanArgs a)
{
    __shared__ unsigned long long s_ec[kScanT];
    __shared__ uint4 s_rm[kScanT];
    const bool out = blockIdx.x >= a.nb_in;
    const uint32_t nb = out ? blockIdx.x - a.nb_in : blockIdx.x;
    const uint32_t n = out ? a.n_out : a.n_in;
    const uint32_t base = nb * (kScanT * I) + threadIdx.x * I;
    unsigned long long ec = 0;
    uint4 rm = make_uint4(0u, 0u, 0u, 0u);
    int32_t rows[I];
    uint32_t cs[I];
    scan_items<K, BATCH, I>(a, out, base, n, rows, cs);
#pragma unroll
    for (int k = 0; k < I; ++k) {
        if (rows[k] >= 0) {
            ec += pack_ec(cs[k], out);
            rm = add4(rm, split_counts(cs[k], out));
        }
    }
    s_ec[threadIdx.x] = ec;
    s_rm[threadIdx.x] = rm;
    __syncthreads();
    for (int s = kScanT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s_ec[threadIdx.x] += s_ec[threadIdx.x + s];
            s_rm[threadIdx.x] = add4(s_rm[threadIdx.x], s_rm[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.part_ec[blockIdx.x] = s_ec[0];
        a.part_rm[blockIdx.x] = s_rm[0];
    }
}

template <int K, bool BATCH, int I>
__global__ __launch_bounds__(256) void sgns_scan_write(ScanArgs a)
{
    __shared__ unsigned long long s_ec[kScanT];
    __shared__ uint4 s_rm[kScanT];
    const bool out = blockIdx.x >= a.nb_in;
    const uint32_t b0 = out ? a.nb_in : 0u;   // first block of this table
    const uint32_t n = out ? a.n_out : a.n_in;
    const uint32_t nb = blockIdx.x - b0;
    // offset of this block: partials of the earlier blocks of the same table
    unsigned long long pre = 0;
    uint4 pre_rm = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t b = b0 + threadIdx.x; b < blockIdx.x; b += kScanT) {
        pre += a.part_ec[b];
        pre_rm = add4(pre_rm, a.part_rm[b]);
    }
    s_ec[threadIdx.x] = pre;
    s_rm[threadIdx.x] = pre_rm;
    __syncthreads();
    for (int s = kScanT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s_ec[threadIdx.x] += s_ec[threadIdx.x + s];
            s_rm[threadIdx.x] = add4(s_rm[threadIdx.x], s_rm[threadIdx.x + s]);
        }
        __syncthreads();
    }
    const unsigned long long blk_ec = s_ec[0];
    const uint4 blk_rm = s_rm[0];
    __syncthreads();

    const uint32_t base = nb * (kScanT * I) + threadIdx.x * I;
    // (entries scanned in the low word; the chunk count in the high word is unused here)
    int32_t rows[I];
    uint32_t cs[I];
    unsigned long long mine = 0;
    uint4 mine_rm = make_uint4(0u, 0u, 0u, 0u);
    scan_items<K, BATCH, I>(a, out, base, n, rows, cs);
#pragma unroll
    for (int k = 0; k < I; ++k) {
        if (rows[k] >= 0) {
            mine += pack_ec(cs[k], out);
            mine_rm = add4(mine_rm, split_counts(cs[k], out));
        }
    }
    // block exclusive scans
    s_ec[threadIdx.x] = mine;
    s_rm[threadIdx.x] = mine_rm;
    __syncthreads();
    for (int off = 1; off < kScanT; off <<= 1) {
        const unsigned long long add = threadIdx.x >= off ? s_ec[threadIdx.x - off] : 0ull;
        const uint4 add_rm = threadIdx.x >= off ? s_rm[threadIdx.x - off] : make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();
        s_ec[threadIdx.x] += add;
        s_rm[threadIdx.x] = add4(s_rm[threadIdx.x], add_rm);
        __syncthreads();
    }
    const unsigned long long run = blk_ec + s_ec[threadIdx.x] - mine;
    const uint4 at = s_rm[threadIdx.x];
    uint32_t slot = blk_rm.x + at.x - mine_rm.x;    // list slot
    uint32_t mrow = blk_rm.y + at.y - mine_rm.y;    // split-row index
    uint32_t mchunk = blk_rm.z + at.z - mine_rm.z;  // first chunk of the next split row
    uint32_t sgl = blk_rm.w + at.w - mine_rm.w;     // single-touch out rows before
    uint32_t entry = (uint32_t)run;
    int32_t* list = out ? a.list_out : a.list_in;
    int32_t* off = out ? a.off_out : a.off_in;
    int4* chunks = out ? a.chunks_out : a.chunks_in;   // one per row of at most kChunk touches
    int4* split = out ? a.split_out : a.split_in;      // chunks of the split rows
    int4* mrows = out ? a.mrows_out : a.mrows_in;
#pragma unroll
    for (int k = 0; k < I; ++k) {
        if (rows[k] >= 0) {
            const uint32_t c = cs[k];
            list[slot] = rows[k];
            if (single_out(c, out)) {
                // the forward adds this row's delta; -1 - slot marks it and
                // carries its list slot
                off[rows[k]] = -1 - (int32_t)slot;
                if (a.reset) a.cnt_out[rows[k]] = 0u;
                ++sgl;
            } else {
                const uint32_t nch = (c + kChunk - 1) / kChunk;
                off[rows[k]] = (int32_t)entry;
                if (nch == 1) {
                    chunks[slot - mrow - sgl] =
                        make_int4(rows[k], (int32_t)entry, (int32_t)c, (int32_t)slot);
                } else {
                    mrows[mrow] = make_int4(rows[k], (int32_t)mchunk, (int32_t)nch, (int32_t)slot);
                    for (uint32_t j = 0; j < nch; ++j)
                        split[mchunk + j] = make_int4(rows[k], (int32_t)(entry + j * kChunk),
                                                      (int32_t)min((uint32_t)kChunk, c - j * kChunk),
                                                      (int32_t)(mchunk + j));
                    ++mrow;
                    mchunk += nch;
                }
                entry += c;
            }
            ++slot;
        }
        if (base + k + 1 == n) {   // the table's last item: totals
            a.meta[out ? 1 : 0] = slot;
            a.meta[out ? 3 : 2] = slot - mrow - sgl;   // rows of one chunk
            a.meta[out ? 5 : 4] = mrow;          // split rows
            a.meta[out ? 7 : 6] = mchunk;        // their chunks
        }
    }
}

// ---------------------------------------------------------------- forward
struct FwdArgs {
    const float* __restrict__ tin;
    float* __restrict__ tout;      // single-touch out rows are updated here
    const int32_t* __restrict__ touch_row;
    const uint32_t* __restrict__ touch_pos;
    const int32_t* __restrict__ off_in;
    const int32_t* __restrict__ off_out;
    uint32_t npairs;
    int32_t ppw;             // pairs per wave, ppw (K + 2) <= 64
    float lr;
    int4* ent_out;           // (FP64 g, ctx, pair-order key p (K+1) + k) by out-row
                             // segment position
    float* dinp;             // [P][d] sum_k g_k out[t_k] (FP64 sum, rounded once) by
                             // in-row segment position
    uint32_t* key_in;        // the pair p, same position
    double* loss_part;       // one slot per wave
    float* cap_out;          // capture != NULL: single-touch out-row deltas to cap_out[slot][d]
};

// One pair per group of LPP lanes, 64 / LPP pairs at a time.  With FP64
// dots and coefficients the kernel needs 164 registers at d = 128, K = 5
// (three waves per SIMD).
template <int D, int K>
__global__ __launch_bounds__(256) void sgns_forward_kernel(FwdArgs a)
{
    constexpr int LPP = fwd_lanes_per_pair<D, K>();   // lanes per pair
    constexpr int G = 64 / LPP;               // pairs in flight per wave
    constexpr int V4 = D / (4 * LPP);         // float4s per lane and row
    constexpr int T = K + 2;                  // touches per pair
    const int lane = threadIdx.x & 63;
    const int grp = lane / LPP, gl = lane % LPP;
    const uint32_t gwave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t q0 = gwave * (uint32_t)a.ppw;
    if (q0 >= a.npairs) return;
    const int np = (int)min((uint32_t)a.ppw, a.npairs - q0);

    // ---- touch metadata: lane l < np T holds touch l of the wave's pairs and
    //      its position in its row's segment, or, for an out row touched once
    //      in the minibatch, the row's list slot (and a bit in `single`)
    int32_t m_row = -1;
    uint32_t m_pos = 0;
    bool m_single = false;
    if (lane < np * T) {
        const uint32_t t = q0 * T + lane;
        m_row = a.touch_row[t];
        const uint32_t rk = a.touch_pos[t];
        const bool in = (lane % T) == 0;
        if (m_row >= 0) {
            const int32_t off = (in ? a.off_in : a.off_out)[m_row];
            m_single = off < 0;
            m_pos = m_single ? (uint32_t)(-1 - off) : (uint32_t)off + rk;
        }
    }
    const unsigned long long single = __ballot(m_single);

    double lacc = 0.0;
    for (int base = 0; base < np; base += G) {
        const int p = base + grp;
        const bool live = p < np;
        const uint32_t q = q0 + (uint32_t)p;   // pair index within the minibatch
        const int src = (live ? p : 0) * T;
        const int32_t ctx = __shfl(m_row, src);
        const uint32_t pos_in = __shfl(m_pos, src);
        int32_t t[K + 1];
#pragma unroll
        for (int k = 0; k <= K; ++k) t[k] = __shfl(m_row, src + 1 + k);
        // out position of touch k = gl (and, with 16 lanes, k = gl + 16)
        const uint32_t my_pos = __shfl(m_pos, src + 1 + (gl <= K ? gl : 0));
        uint32_t my_pos_hi = 0;
        if (LPP == 16 && K >= 16) my_pos_hi = __shfl(m_pos, src + 1 + (gl + 16 <= K ? gl + 16 : 0));

        float4 vin[V4];
        float4 vo[K + 1][V4];
        const float4* ri = row4<D>(a.tin, live ? ctx : 0);
#pragma unroll
        for (int i = 0; i < V4; ++i) vin[i] = ri[i * LPP + gl];
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            const bool ok = live && t[k] >= 0;
            const float4* ro = row4<D>(a.tout, ok ? t[k] : 0);
#pragma unroll
            for (int i = 0; i < V4; ++i)
                vo[k][i] = ok ? ro[i * LPP + gl] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        // dots, sigma and coefficients in FP64 over the FP32 entries; lane
        // k mod LPP of the group takes touch k's loss term, -log sigma(s0) for
        // the centre and -log sigma(-s_k) for a negative
        const double lr = (double)a.lr;
        double g[K + 1];
        coefficients<K, LPP, V4>(vin, vo, t, lr, live, gl, grp, g, lacc);

        // lane j of the group writes the entry of touch k = j (and j + 16)
#pragma unroll
        for (int h = 0; h < (K + LPP) / LPP; ++h) {
            const int k = gl + h * LPP;
            double gk = g[0];
            int32_t tk = t[0];
#pragma unroll
            for (int j = 1; j <= K; ++j)
                if (k == j) {
                    gk = g[j];
                    tk = t[j];
                }
            if (k <= K && live && tk >= 0 && !((single >> (src + 1 + k)) & 1ull)) {
                const uint32_t pos = h == 0 ? my_pos : my_pos_hi;
                store_nt(&a.ent_out[pos], pack_entry(gk, ctx, q * (K + 1) + (uint32_t)k));
            }
        }
        // out rows touched once: row + g in[ctx] in FP64, rounded once (or the
        // delta alone, when capturing)
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            uint32_t slot = 0;
            if (a.cap_out) slot = __shfl(m_pos, src + 1 + k);   // uniform branch
            if (live && t[k] >= 0 && ((single >> (src + 1 + k)) & 1ull)) {
                float4* dst = reinterpret_cast<float4*>(
                    a.cap_out ? a.cap_out + (int64_t)slot * D : a.tout + (int64_t)t[k] * D);
#pragma unroll
                for (int i = 0; i < V4; ++i) {
                    const float4 base = a.cap_out ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : vo[k][i];
                    const float4 d = make_float4(
                        (float)fma(g[k], (double)vin[i].x, (double)base.x),
                        (float)fma(g[k], (double)vin[i].y, (double)base.y),
                        (float)fma(g[k], (double)vin[i].z, (double)base.z),
                        (float)fma(g[k], (double)vin[i].w, (double)base.w));
                    store_nt(&dst[i * LPP + gl], d);
                }
            }
        }
        if (live) {
            if (gl == 0) store_nt(&a.key_in[pos_in], q);
            float4* dp = reinterpret_cast<float4*>(a.dinp + (int64_t)pos_in * D);
#pragma unroll
            for (int i = 0; i < V4; ++i) {
                double ax = 0.0, ay = 0.0, az = 0.0, aw = 0.0;
#pragma unroll
                for (int k = 0; k <= K; ++k) {
                    ax = fma(g[k], (double)vo[k][i].x, ax);
                    ay = fma(g[k], (double)vo[k][i].y, ay);
                    az = fma(g[k], (double)vo[k][i].z, az);
                    aw = fma(g[k], (double)vo[k][i].w, aw);
                }
                store_nt(&dp[i * LPP + gl], make_float4((float)ax, (float)ay, (float)az, (float)aw));
            }
        }
    }
    lacc = wave_sum_f64(lacc);
    if (lane == 0) a.loss_part[gwave] += lacc;
}

// ---------------------------------------------------------------- reduce
// Out rows: delta out[t] = sum over touches of g * in[ctx].
// In rows:  delta in[c]  = sum over touches of the pair's in-row delta.
// Rows of at most kChunk touches: one 16-lane group per row sorts the
// touches by their pair-order key (a bitonic network over the group) and
// sums their FP64 terms in that order, so the result is the sequential sum
// in pair order whatever the atomics did.  Chunks of the rows with more
// touches (their membership follows the atomics' order) get exact sums
// instead, which a merge adds in chunk order.
// Sort (key, a, b) ascending over the 16 lanes of a group.
__device__ __forceinline__ void sort16(uint32_t& key, double& va, int32_t& vb, int gl)
{
#pragma unroll
    for (int k = 2; k <= 16; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t pk = __shfl_xor(key, j);
            const double pa = __shfl_xor(va, j);
            const int32_t pb = __shfl_xor(vb, j);
            const bool up = (gl & k) == 0;        // this pair of lanes sorts ascending
            const bool low = (gl & j) == 0;       // this lane keeps the smaller key
            const bool take = (low == up) ? pk < key : pk > key;
            if (take) {
                key = pk;
                va = pa;
                vb = pb;
            }
        }
}

// Two launches per minibatch, each over a list of work items of three kinds:
//   first:  chunks of split out rows, chunks of split in rows (exact sums,
//           stored), out rows of at most kChunk touches (sorted FP32 sums);
//   second: in rows of at most kChunk touches, then the merge of the split
//           out rows and split in rows (their chunks' sums in chunk order).
// Out rows need the in-table as of the minibatch start, so every in row is
// written in the second launch.
struct ApplyArgs {
    float* tin;
    float* tout;
    const int4* ent_out;          // (FP64 g, ctx, pair-order key) by out segment position
    const float* dinp;            // in-row delta of each pair, by in segment position
    const uint32_t* key_in;       // pair by in segment position
    const int4* chunks_in;        // rows of at most kChunk touches
    const int4* chunks_out;
    const int4* split_in;         // chunks of split rows
    const int4* split_out;
    const int4* mrows_in;         // split rows
    const int4* mrows_out;
    double* partial_in;           // exact sums of the split rows' chunks
    double* partial_out;
    uint32_t* cnt_in;
    uint32_t* cnt_out;
    const uint32_t* meta;         // this minibatch's counters
    float* cap_in;                // capture != NULL: deltas to capture[list slot][d]
    float* cap_out;
    unsigned long long* row_totals;
    double grid_c;                // 1.5 * 2^(floor(log2 lr) + 17)
    int32_t reset;                // zero the counters of the rows done here
};

template <int D, int PHASE>
__global__ __launch_bounds__(256) void sgns_apply_kernel(ApplyArgs a)
{
    constexpr int V4 = D / 64;
    // rows in flight per group, rows of one chunk: fewer registers and more
    // waves beat more loads per wave here (65,536 pairs on R-MAT 2^20, us per
    // minibatch with 4 / 2 / 1 rows: d = 64 128.4 / 124.7 / 125.9, d = 128
    // 193.9 / 184.6 / 180.2, d = 256 400.8 / 346.3 / 319.1)
    constexpr int kRows = D >= 128 ? 1 : 2;
    constexpr int kRowsS = 2;   // rows in flight per group, chunks of split rows
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, gl = lane & 15;
    const int g0 = grp << 4;
    // item ranges [0, e1) [e1, e2) [e2, e3)
    const uint32_t e1 = PHASE == 0 ? a.meta[7] : a.meta[2];
    const uint32_t e2 = e1 + (PHASE == 0 ? a.meta[6] : a.meta[5]);
    const uint32_t e3 = e2 + (PHASE == 0 ? a.meta[3] : a.meta[4]);
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    // the descriptor of item c: a chunk of a split row, a row of one chunk, or
    // a split row to merge
    auto desc_of = [&](uint32_t c) -> int4 {
        const int kind = c < e1 ? 0 : (c < e2 ? 1 : 2);
        const uint32_t ci = kind == 0 ? c : (kind == 1 ? c - e1 : c - e2);
        const int4* arr = PHASE == 0
            ? (kind == 0 ? a.split_out : (kind == 1 ? a.split_in : a.chunks_out))
            : (kind == 0 ? a.chunks_in : (kind == 1 ? a.mrows_out : a.mrows_in));
        return arr[ci];
    };
    const uint32_t stride = nw * 4u;
    const uint32_t first = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 4u;
    int4 next = first + grp < e3 ? desc_of(first + grp) : make_int4(0, 0, 0, 0);
    for (uint32_t base = first; base < e3; base += stride) {
        const uint32_t c = base + grp;
        const int4 d = next;
        // the next item's descriptor is in flight while this one is done
        if (c + stride < e3) next = desc_of(c + stride);
        if (c >= e3) continue;
        const int kind = c < e1 ? 0 : (c < e2 ? 1 : 2);
        if (PHASE == 1 && kind > 0) {
            // merge of a split row: its chunks' exact sums in chunk order
            const bool out = kind == 1;
            const int4 m = d;
            float4 cur[V4];
            get_row<D>(out ? a.tout : a.tin, out ? a.cap_out : a.cap_in, m.x, cur, gl);
            const double* partial = out ? a.partial_out : a.partial_in;
            double acc[D / 16];
#pragma unroll
            for (int e = 0; e < D / 16; ++e) acc[e] = 0.0;
            for (int32_t j = 0; j < m.z; ++j) {
                const double* pr = partial + (int64_t)(m.y + j) * D;
#pragma unroll
                for (int i = 0; i < V4; ++i) {
                    const double2* q = reinterpret_cast<const double2*>(pr + (i * 16 + gl) * 4);
                    const double2 u = q[0], v = q[1];
                    acc[4 * i + 0] += u.x;
                    acc[4 * i + 1] += u.y;
                    acc[4 * i + 2] += v.x;
                    acc[4 * i + 3] += v.y;
                }
            }
            put_row<D>(out ? a.tout : a.tin, out ? a.cap_out : a.cap_in, m.x, m.w, cur, acc, gl);
            if (a.reset && gl == 0) (out ? a.cnt_out : a.cnt_in)[m.x] = 0;
            continue;
        }
        // out rows draw on in[ctx] with coefficient g, in rows on the per-pair deltas
        const bool split = PHASE == 0 && kind < 2;
        const bool out = PHASE == 0 ? kind != 1 : false;
        const int32_t row = d.x, start = d.y, len = d.z, slot = d.w;
        const float* src = out ? a.tin : a.dinp;
        double my_g = 1.0;
        int32_t my_src = start + gl;
        uint32_t my_key = 0xffffffffu;
        if (gl < len) {
            if (out) {
                const int4 e = a.ent_out[start + gl];
                my_g = entry_g(e);
                my_src = e.z;
                my_key = (uint32_t)e.w;
            } else {
                my_key = a.key_in[start + gl];
            }
        }
        if (split) {
            // exact sums, stored for the merge
            double acc[D / 16];
#pragma unroll
            for (int e = 0; e < D / 16; ++e) acc[e] = 0.0;
            const double gc = a.grid_c;
            for (int32_t i0 = 0; i0 < len; i0 += kRowsS) {
                double gg[kRowsS];
                float4 x[kRowsS][V4];
#pragma unroll
                for (int u = 0; u < kRowsS; ++u) {
                    const int32_t idx = min(i0 + u, kChunk - 1);
                    const bool ok = i0 + u < len;
                    gg[u] = ok ? __shfl(my_g, g0 + idx) : 0.0;
                    const int32_t rr = __shfl(my_src, g0 + idx);
                    const float4* rp = row4<D>(src, ok ? rr : 0);
#pragma unroll
                    for (int i = 0; i < V4; ++i)
                        x[u][i] = ok ? rp[i * 16 + gl] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                }
#pragma unroll
                for (int u = 0; u < kRowsS; ++u) {
                    // each FP64 term g * x is rounded once more, onto the grid
                    const double gd = gg[u];
#pragma unroll
                    for (int i = 0; i < V4; ++i) {
                        acc[4 * i + 0] += on_grid(gd * (double)x[u][i].x, gc);
                        acc[4 * i + 1] += on_grid(gd * (double)x[u][i].y, gc);
                        acc[4 * i + 2] += on_grid(gd * (double)x[u][i].z, gc);
                        acc[4 * i + 3] += on_grid(gd * (double)x[u][i].w, gc);
                    }
                }
            }
            double* pr = (out ? a.partial_out : a.partial_in) + (int64_t)slot * D;
#pragma unroll
            for (int i = 0; i < V4; ++i) {
                double2* q = reinterpret_cast<double2*>(pr + (i * 16 + gl) * 4);
                q[0] = make_double2(acc[4 * i + 0], acc[4 * i + 1]);
                q[1] = make_double2(acc[4 * i + 2], acc[4 * i + 3]);
            }
            continue;
        }
        // a row of at most kChunk touches: FP64 sum in pair order
        float4 cur[V4];
        get_row<D>(out ? a.tout : a.tin, out ? a.cap_out : a.cap_in, row, cur, gl);
        uint32_t key = my_key;
        sort16(key, my_g, my_src, gl);
        double acc[D / 16];
#pragma unroll
        for (int e = 0; e < D / 16; ++e) acc[e] = 0.0;
        for (int32_t i0 = 0; i0 < len; i0 += kRows) {
            double gg[kRows];
            float4 x[kRows][V4];
#pragma unroll
            for (int u = 0; u < kRows; ++u) {
                const int32_t idx = min(i0 + u, kChunk - 1);
                const bool ok = i0 + u < len;
                gg[u] = __shfl(my_g, g0 + idx);
                const int32_t rr = __shfl(my_src, g0 + idx);
                const float4* rp = row4<D>(src, ok ? rr : 0);
#pragma unroll
                for (int i = 0; i < V4; ++i)
                    x[u][i] = ok ? rp[i * 16 + gl] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < kRows; ++u)
#pragma unroll
                for (int i = 0; i < V4; ++i) {
                    // in rows: g = 1, and 1 * x + acc is exactly x + acc
                    acc[4 * i + 0] = fma(gg[u], (double)x[u][i].x, acc[4 * i + 0]);
                    acc[4 * i + 1] = fma(gg[u], (double)x[u][i].y, acc[4 * i + 1]);
                    acc[4 * i + 2] = fma(gg[u], (double)x[u][i].z, acc[4 * i + 2]);
                    acc[4 * i + 3] = fma(gg[u], (double)x[u][i].w, acc[4 * i + 3]);
                }
        }
        put_row<D>(out ? a.tout : a.tin, out ? a.cap_out : a.cap_in, row, slot, cur, acc, gl);
        if (a.reset && gl == 0) (out ? a.cnt_out : a.cnt_in)[row] = 0;
    }
    // the second launch counts the minibatch's touched rows
    if (PHASE == 1 && blockIdx.x == 0 && threadIdx.x == 0) {
        a.row_totals[0] += a.meta[0];
        a.row_totals[1] += a.meta[1];
        a.row_totals[2] += a.meta[1] - a.meta[3] - a.meta[5];   // out rows touched once
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

void launch_loss_reduce(const double* part, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, s, part, n, out);
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
    const int64_t chunk = chunk_walks_of(p);
    FELOG_REQUIRE(w.chunk_ready.empty() || w.chunk_for_valid == chunk,
                  "the corpus is being written in chunks of %lld walks, not %lld",
                  (long long)w.chunk_for_valid, (long long)chunk);
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

TrainSchedule train_schedule(Walks& w, const felog_train_params& p) { return make_schedule(w, p); }

std::vector<int32_t> train_slices(int32_t L, int32_t window) { return make_slices(L, window); }

int64_t count_minibatches(Walks& w, const felog_train_params& p, int64_t* total_pairs)
{
    TrainSchedule s = make_schedule(w, p);
    if (total_pairs) *total_pairs = s.total_pairs;
    return s.B;
}

void model_alloc_update_state(Model& m)
{
    Ctx& c = *m.ctx;
    const int64_t n = m.g->n;
    for (MinibatchBufs& b : m.mb) {
        b.cnt_in.alloc(&c, sizeof(uint32_t) * n);
        b.cnt_out.alloc(&c, sizeof(uint32_t) * n);
        b.off_in.alloc(&c, sizeof(int32_t) * n);
        b.off_out.alloc(&c, sizeof(int32_t) * n);
        FELOG_HIP(hipMemsetAsync(b.cnt_in.ptr, 0, sizeof(uint32_t) * n, c.stream));
        FELOG_HIP(hipMemsetAsync(b.cnt_out.ptr, 0, sizeof(uint32_t) * n, c.stream));
    }
    m.meta.alloc(&c, sizeof(uint32_t) * kIdSets * kMetaWords);
    m.row_totals.alloc(&c, sizeof(uint64_t) * 3);
    m.loss_out.alloc(&c, sizeof(double));
    FELOG_HIP(hipMemsetAsync(m.meta.ptr, 0, m.meta.bytes, c.stream));
}

// Rows split over chunks have more than kChunk touches, so at most
// touches / (kChunk + 1) of them, with ceil(c / kChunk) <= 2 c / (kChunk + 1)
// chunks each: at most touches / 8 + 1 chunks in all.
static int64_t max_split_rows(int64_t touches) { return touches / (kChunk + 1) + 1; }

// Largest minibatch whose launches all go to the training stream.
constexpr int64_t kOneStreamPairs = 2048;
// Zero the row counters whole when n <= this many times the minibatch's touches.
constexpr int64_t kZeroWholeRatio = 8;
static int64_t max_split_chunks(int64_t touches) { return touches / 8 + 1; }

// Launch geometry and per-minibatch values of one minibatch.
struct MinibatchLaunch {
    uint32_t npairs;
    int dim, K;
    uint32_t prep_blocks, fwd_blocks, nb_in, nb_out, reduce_blocks;
    int scan_i;           // scan items per thread (kScanISmall or kScanILarge)
    int64_t split_in;     // partial-sum rows reserved for the in-table (the out-table's follow)
    double grid_c;        // exact-sum grid constant of this minibatch's learning rate
    bool one_stream;      // ids on the training stream (on the critical path)
    bool zero_whole;      // zero the row counters whole before the ids (else reset rows)
};

// Zeroes a[0, n) and b[0, n): 16-byte stores, then the tails.
__global__ __launch_bounds__(256) void zero_counters_kernel(uint32_t* a, uint32_t* b, int64_t n)
{
    const int64_t n4 = n / 4;
    const int64_t stride = (int64_t)gridDim.x * 256;
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 2 * n4; i += stride) {
        uint4* p = reinterpret_cast<uint4*>(i < n4 ? a : b);
        p[i < n4 ? i : i - n4] = z;
    }
    if (blockIdx.x == 0 && threadIdx.x < (int)(n - 4 * n4)) {
        a[4 * n4 + threadIdx.x] = 0u;
        b[4 * n4 + threadIdx.x] = 0u;
    }
}

static void zero_counters(MinibatchBufs& mb, hipStream_t s)
{
    const int64_t n = (int64_t)(mb.cnt_in.bytes / sizeof(uint32_t));
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n / 2 + 255) / 256, 512));
    hipLaunchKernelGGL(zero_counters_kernel, dim3(blocks), dim3(256), 0, s,
                       mb.cnt_in.as<uint32_t>(), mb.cnt_out.as<uint32_t>(), n);
}

// When the ids run on a second stream and the table is not much larger than
// the minibatch's touches, the row counters are zeroed whole before each
// minibatch's ids (two streaming writes of n words beside the training
// launches) instead of with one scattered write per touched row on the
// training stream; otherwise the rows are reset as they are done.
// Ids, ranks and the destination sort of one minibatch (reads only the walks
// and the noise table, so it may run ahead of the training of earlier ones).
template <int K>
static void launch_ids_t(MinibatchBufs& mb, PrepArgs pa, const MinibatchLaunch& ml,
                         uint32_t* meta, hipStream_t s)
{
    if (ml.zero_whole) zero_counters(mb, s);
    pa.cnt_in = mb.cnt_in.as<uint32_t>();
    pa.cnt_out = mb.cnt_out.as<uint32_t>();
    pa.touch_row = mb.touch_row.as<int32_t>();
    pa.touch_pos = mb.touch_pos.as<uint32_t>();
    hipLaunchKernelGGL((sgns_prep_kernel<K>), dim3(ml.prep_blocks), dim3(256), 0, s, pa);
    const uint32_t nb = ml.nb_in + ml.nb_out;
    uint4* part_rm = mb.partials.as<uint4>();
    unsigned long long* part_ec = reinterpret_cast<unsigned long long*>(part_rm + nb);
    ScanArgs sa{pa.touch_row, pa.touch_pos, pa.cnt_in, pa.cnt_out, ml.npairs,
                ml.npairs * (uint32_t)(K + 1), ml.nb_in, part_ec, part_rm,
                mb.list_in.as<int32_t>(), mb.list_out.as<int32_t>(), mb.off_in.as<int32_t>(),
                mb.off_out.as<int32_t>(), mb.chunks_in.as<int4>(), mb.chunks_out.as<int4>(),
                mb.split_in.as<int4>(), mb.split_out.as<int4>(), mb.mrows_in.as<int4>(),
                mb.mrows_out.as<int4>(), meta, ml.zero_whole ? 0 : 1};
    const bool small = ml.scan_i == kScanISmall;
    if (ml.one_stream && small) {
        hipLaunchKernelGGL((sgns_scan_partials<K, true, kScanISmall>), dim3(nb), dim3(256), 0, s, sa);
        hipLaunchKernelGGL((sgns_scan_write<K, true, kScanISmall>), dim3(nb), dim3(256), 0, s, sa);
    } else if (ml.one_stream) {
        hipLaunchKernelGGL((sgns_scan_partials<K, true, kScanILarge>), dim3(nb), dim3(256), 0, s, sa);
        hipLaunchKernelGGL((sgns_scan_write<K, true, kScanILarge>), dim3(nb), dim3(256), 0, s, sa);
    } else if (small) {
        hipLaunchKernelGGL((sgns_scan_partials<K, false, kScanISmall>), dim3(nb), dim3(256), 0, s, sa);
        hipLaunchKernelGGL((sgns_scan_write<K, false, kScanISmall>), dim3(nb), dim3(256), 0, s, sa);
    } else {
        hipLaunchKernelGGL((sgns_scan_partials<K, false, kScanILarge>), dim3(nb), dim3(256), 0, s, sa);
        hipLaunchKernelGGL((sgns_scan_write<K, false, kScanILarge>), dim3(nb), dim3(256), 0, s, sa);
    }
    FELOG_HIP(hipGetLastError());
}

// Forward and the two apply launches of one minibatch whose ids are ready.
// ev (optional): [0] recorded before the forward, [1] after it, [2] after the
// first apply launch, [3] at the end;
// fwd_done (optional) is recorded after the forward.
template <int D, int K>
static void launch_train_t(Model& m, MinibatchBufs& mb, FwdArgs fa, const MinibatchLaunch& ml,
                           uint32_t* meta, float* cap_in, float* cap_out, hipStream_t s,
                           hipEvent_t* ev, hipEvent_t fwd_done)
{
    fa.touch_row = mb.touch_row.as<int32_t>();
    fa.touch_pos = mb.touch_pos.as<uint32_t>();
    fa.off_in = mb.off_in.as<int32_t>();
    fa.off_out = mb.off_out.as<int32_t>();
    fa.cap_out = cap_out;
    if (ev) FELOG_HIP(hipEventRecord(ev[0], s));
    hipLaunchKernelGGL((sgns_forward_kernel<D, K>), dim3(ml.fwd_blocks), dim3(256), 0, s, fa);
    if (ev) FELOG_HIP(hipEventRecord(ev[1], s));
    if (fwd_done) FELOG_HIP(hipEventRecord(fwd_done, s));
    double* part_in = m.partial.as<double>();
    double* part_out = part_in + ml.split_in * D;
    ApplyArgs aa{m.tin.as<float>(),       m.tout.as<float>(),      fa.ent_out,
                 fa.dinp,                 fa.key_in,
                 mb.chunks_in.as<int4>(), mb.chunks_out.as<int4>(), mb.split_in.as<int4>(),
                 mb.split_out.as<int4>(), mb.mrows_in.as<int4>(),  mb.mrows_out.as<int4>(),
                 part_in,                 part_out,                mb.cnt_in.as<uint32_t>(),
                 mb.cnt_out.as<uint32_t>(), meta,                  cap_in,
                 cap_out,                 m.row_totals.as<unsigned long long>(), ml.grid_c,
                 ml.zero_whole ? 0 : 1};
    hipLaunchKernelGGL((sgns_apply_kernel<D, 0>), dim3(ml.reduce_blocks), dim3(256), 0, s, aa);
    if (ev) FELOG_HIP(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL((sgns_apply_kernel<D, 1>), dim3(ml.reduce_blocks), dim3(256), 0, s, aa);
    if (ev) FELOG_HIP(hipEventRecord(ev[3], s));
    FELOG_HIP(hipGetLastError());
}

#define FELOG_FOR_K(X)                                                               \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) \
    X(16) X(17) X(18) X(19) X(20)

static void launch_ids(MinibatchBufs& mb, const PrepArgs& pa, const MinibatchLaunch& ml,
                       uint32_t* meta, hipStream_t s)
{
    switch (ml.K) {
#define FELOG_CASE(k)                                  \
    case k:                                            \
        launch_ids_t<k>(mb, pa, ml, meta, s);          \
        break;
        FELOG_FOR_K(FELOG_CASE)
#undef FELOG_CASE
        default: fail(FELOG_EUNSUPPORTED, "negatives = %d not supported", ml.K);
    }
}

template <int D>
static void launch_train_d(Model& m, MinibatchBufs& mb, const FwdArgs& fa,
                           const MinibatchLaunch& ml, uint32_t* meta, float* ci, float* co,
                           hipStream_t s, hipEvent_t* ev, hipEvent_t fd)
{
    switch (ml.K) {
#define FELOG_CASE(k)                                                      \
    case k:                                                                \
        launch_train_t<D, k>(m, mb, fa, ml, meta, ci, co, s, ev, fd);      \
        break;
        FELOG_FOR_K(FELOG_CASE)
#undef FELOG_CASE
        default: fail(FELOG_EUNSUPPORTED, "negatives = %d not supported", ml.K);
    }
}

static void launch_train(Model& m, MinibatchBufs& mb, const FwdArgs& fa,
                         const MinibatchLaunch& ml, uint32_t* meta, float* ci, float* co,
                         hipStream_t s, hipEvent_t* ev, hipEvent_t fd = nullptr)
{
    if (ml.dim == 64) launch_train_d<64>(m, mb, fa, ml, meta, ci, co, s, ev, fd);
    else if (ml.dim == 128) launch_train_d<128>(m, mb, fa, ml, meta, ci, co, s, ev, fd);
    else launch_train_d<256>(m, mb, fa, ml, meta, ci, co, s, ev, fd);
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
        FELOG_REQUIRE(cnt <= ((int64_t)1 << 31), "delta capture of a BF16 model is limited to "
                      "n * d <= 2^31");
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

    if (apply && small_path_applies(m, p)) {
        std::vector<int32_t> sl = make_slices(w.L, p.window);
        DevBuf slices;
        slices.alloc(&c, sizeof(int32_t) * std::max<size_t>(sl.size(), 1));
        if (!sl.empty())
            FELOG_HIP(hipMemcpyAsync(slices.ptr, sl.data(), sizeof(int32_t) * sl.size(),
                                     hipMemcpyHostToDevice, c.stream));
        train_minibatches_small(m, w, p, sch, slices.as<int32_t>(), first_mb, end, stats);
        return;
    }

    // scratch sized for this minibatch size
    if (m.cap_pairs < P || m.cap_K < K) {
        m.cap_pairs = std::max<int64_t>(m.cap_pairs, P);
        m.cap_K = std::max(m.cap_K, K);
        const int64_t cp = m.cap_pairs, ck = m.cap_K;
        const int64_t touches_out = cp * (ck + 1);
        const int64_t nbmax = (cp + kScanSpanMin - 1) / kScanSpanMin +
                              (touches_out + kScanSpanMin - 1) / kScanSpanMin;
        for (MinibatchBufs& b : m.mb) {
            b.touch_row.alloc(&c, sizeof(int32_t) * cp * (ck + 2));
            b.touch_pos.alloc(&c, sizeof(uint32_t) * cp * (ck + 2));
            b.list_in.alloc(&c, sizeof(int32_t) * cp);
            b.list_out.alloc(&c, sizeof(int32_t) * touches_out);
            b.chunks_in.alloc(&c, sizeof(int4) * cp);
            b.chunks_out.alloc(&c, sizeof(int4) * touches_out);
            b.split_in.alloc(&c, sizeof(int4) * max_split_chunks(cp));
            b.split_out.alloc(&c, sizeof(int4) * max_split_chunks(touches_out));
            b.mrows_in.alloc(&c, sizeof(int4) * max_split_rows(cp));
            b.mrows_out.alloc(&c, sizeof(int4) * max_split_rows(touches_out));
            b.partials.alloc(&c, (sizeof(uint4) + sizeof(unsigned long long)) * nbmax);
        }
        m.ent_out.alloc(&c, sizeof(int4) * touches_out);
        m.dinp.alloc(&c, sizeof(float) * cp * m.dim);
        m.key_in.alloc(&c, sizeof(uint32_t) * cp);
        m.split_rows_in = max_split_chunks(cp);
        m.partial.alloc(&c, sizeof(double) * (m.split_rows_in + max_split_chunks(touches_out)) *
                                m.dim);
    }
    // pairs per forward wave: 4 (more, shorter waves) ran 1.4 us per minibatch
    // faster than 8 at 65,536 pairs, d = 128, K = 5
    const int ppw_max = std::max(1, std::min(4, 64 / (K + 2)));
    const int ppw = (int)std::min<int64_t>(ppw_max,
                                           std::max<int64_t>(1, P / ((int64_t)c.num_cus * 32)));
    const int64_t waves = (P + ppw - 1) / ppw;
    const int64_t blocks = (waves + 3) / 4;
    DevBuf loss_part;
    loss_part.alloc(&c, sizeof(double) * blocks * 4);
    FELOG_HIP(hipMemsetAsync(loss_part.ptr, 0, sizeof(double) * blocks * 4, c.stream));
    FELOG_HIP(hipMemsetAsync(m.row_totals.ptr, 0, sizeof(uint64_t) * 3, c.stream));

    std::vector<int32_t> sl = make_slices(w.L, p.window);
    DevBuf slices;
    slices.alloc(&c, sizeof(int32_t) * std::max<size_t>(sl.size(), 1));
    if (!sl.empty())
        FELOG_HIP(hipMemcpyAsync(slices.ptr, sl.data(), sizeof(int32_t) * sl.size(),
                                 hipMemcpyHostToDevice, c.stream));

    PrepArgs pa{};
    pa.walks = w.data.as<int32_t>();
    pa.W = w.W;
    pa.slices = slices.as<int32_t>();
    pa.id_base = w.id_base;
    pa.window = p.window;
    pa.seed = p.seed;
    pa.noise = NoiseTable{m.cdf.as<uint64_t>(), m.guide.as<int32_t>(), m.total_weight,
                          m.guide_bits};

    FwdArgs fa{};
    fa.tin = m.tin.as<float>();
    fa.tout = m.tout.as<float>();
    fa.ppw = ppw;
    fa.ent_out = m.ent_out.as<int4>();
    fa.dinp = m.dinp.as<float>();
    fa.key_in = m.key_in.as<uint32_t>();
    fa.loss_part = loss_part.as<double>();

    const double lr0 = (double)p.lr_start, lr1 = (double)p.lr_end;
    // Small minibatches run everything on one stream: their launches are
    // chains of a few dependent loads each, and waiting on another stream's
    // events costs more than the overlap gains.
    const bool one_stream = P <= kOneStreamPairs;
    const bool zero_whole = !one_stream && (int64_t)m.g->n <= kZeroWholeRatio * P * (K + 2);
    // minibatches that reset their rows expect zero counters and leave them
    // zero; the others zero them first and leave them dirty
    if (!zero_whole && m.counters_dirty) {
        for (MinibatchBufs& b : m.mb) zero_counters(b, c.stream);
        m.counters_dirty = false;
    }
    if (zero_whole) m.counters_dirty = true;
    // the launch values of minibatch b
    size_t chunk = 0;
    size_t gated = 0;   // walk chunks [0, gated) are known to be written
    auto frame = [&](int64_t b, MinibatchLaunch& ml, PrepArgs& a) {
        while (chunk + 1 < sch.chunk_first_mb.size() && sch.chunk_first_mb[chunk + 1] <= b) ++chunk;
        const int64_t first = (b - sch.chunk_first_mb[chunk]) * P;
        const int64_t np = std::min<int64_t>(P, sch.chunk_pairs[chunk] - first);
        a.vcols = w.valid_cols.as<int32_t>() + sch.chunk_valid_base[chunk];
        a.Wv = (uint32_t)w.chunk_valid[chunk];
        a.first_pair = (uint32_t)first;
        a.npairs = (uint32_t)np;
        ml = MinibatchLaunch{};
        ml.dim = m.dim;
        ml.K = K;
        ml.npairs = (uint32_t)np;
        ml.prep_blocks = (uint32_t)std::min<int64_t>((int64_t)c.num_cus * 4, (np * (K + 2) + 255) / 256);
        ml.fwd_blocks = (uint32_t)(((np + ppw - 1) / ppw + 3) / 4);
        ml.scan_i = P <= kScanSmallPairs ? kScanISmall : kScanILarge;
        const int64_t span = (int64_t)kScanT * ml.scan_i;
        ml.nb_in = (uint32_t)((np + span - 1) / span);
        ml.nb_out = (uint32_t)((np * (K + 1) + span - 1) / span);
        // 16 blocks per CU (faster than 6, 8 or 32 at 65,536 pairs on 2^20 rows),
        // but no more than the items can use: at most one row per touch and per
        // table row, plus the chunks of split rows, 16 items per block at a time
        const int64_t touches = np * (K + 2);
        const int64_t items = std::min<int64_t>(touches, 2 * (int64_t)m.g->n) + touches / kChunk + 16;
        ml.reduce_blocks = (uint32_t)std::max<int64_t>(
            1, std::min<int64_t>((int64_t)c.num_cus * 16, (items + 15) / 16));
        ml.split_in = m.split_rows_in;
        ml.one_stream = one_stream;
        ml.zero_whole = zero_whole;
        const double lr = lr0 - (lr0 - lr1) * (double)b / (double)std::max<int64_t>(1, sch.B - 1);
        const float lr32 = (float)lr;
        ml.grid_c = lr32 > 0.0f ? std::ldexp(1.5, std::ilogb(lr32) + 17) : 1.5;
        return lr32;
    };
    uint32_t* meta0 = m.meta.as<uint32_t>();
    // stream s reads the walks of chunk ch next: wait until they are written
    auto gate = [&](hipStream_t s, size_t ch) {
        while (gated <= ch && gated < w.chunk_ready.size())
            FELOG_HIP(hipStreamWaitEvent(s, w.chunk_ready[gated++], 0));
    };

    // sampled timing: [0] before the ids (on the id stream), [1] after them,
    // [2] before the forward, [3] after it, [4] after the first apply launch,
    // [5] after the second
    const int every = apply ? c.timing_every : 0;
    const size_t pool = c.timing_pool.size() / kTimingEvents;
    size_t next_slot = 0, used_slots = 0;
    int64_t timed = 0;
    double ms_prep = 0.0, ms_fwd = 0.0, ms_apply = 0.0, ms_apply_first = 0.0;
    auto harvest = [&](size_t slot) {
        hipEvent_t* e = &c.timing_pool[kTimingEvents * slot];
        FELOG_HIP(hipEventSynchronize(e[5]));
        float a0 = 0.0f, f = 0.0f, ap = 0.0f, ap0 = 0.0f;
        FELOG_HIP(hipEventElapsedTime(&a0, e[0], e[1]));
        FELOG_HIP(hipEventElapsedTime(&f, e[2], e[3]));
        FELOG_HIP(hipEventElapsedTime(&ap, e[3], e[5]));
        FELOG_HIP(hipEventElapsedTime(&ap0, e[3], e[4]));
        ms_prep += a0;
        ms_fwd += f;
        ms_apply += ap;
        ms_apply_first += ap0;
        ++timed;
    };
    hipEvent_t* slot_of[kIdSets] = {};   // timing events of the minibatch of each id set
    auto take_slot = [&](int64_t b) -> hipEvent_t* {
        if (!(every > 0 && pool > 0 && (b - first_mb) % every == 0)) return nullptr;
        if (used_slots == pool) harvest(next_slot);   // reuse the oldest slot
        else ++used_slots;
        hipEvent_t* e = &c.timing_pool[kTimingEvents * next_slot];
        next_slot = (next_slot + 1) % pool;
        return e;
    };

    int64_t pairs_done = 0;
    FELOG_HIP(hipEventRecord(c.ev0, c.stream));
    if (apply && end > first_mb) {
        // ids of minibatches b + 1 and b + 2 on the second stream while b trains
        // on the first (or all in order on the first, for small minibatches)
        hipStream_t ids_s = c.stream;
        if (!one_stream) {
            c.ensure_aux();
            ids_s = c.aux;
            FELOG_HIP(hipEventRecord(c.pipe_ev[0], c.stream));
            FELOG_HIP(hipStreamWaitEvent(ids_s, c.pipe_ev[0], 0));
        }
        MinibatchLaunch mls[kIdSets];
        float lrs[kIdSets];
        hipEvent_t* ready = c.pipe_ev + 1;               // [set] ids ready
        hipEvent_t* freed = c.pipe_ev + 1 + kIdSets;     // [set] buffers free
        hipEvent_t fwd_done = c.pipe_ev[1 + 2 * kIdSets];
        auto issue_ids = [&](int64_t b) {
            const int set = (int)(b % kIdSets);
            PrepArgs a = pa;
            lrs[set] = frame(b, mls[set], a);
            gate(ids_s, chunk);
            // the set's previous minibatch must be done with it
            if (!one_stream && b >= first_mb + kIdSets)
                FELOG_HIP(hipStreamWaitEvent(ids_s, freed[set], 0));
            hipEvent_t* e = take_slot(b);
            slot_of[set] = e;
            if (e) FELOG_HIP(hipEventRecord(e[0], ids_s));
            launch_ids(m.mb[set], a, mls[set], meta0 + kMetaWords * set, ids_s);
            if (e) FELOG_HIP(hipEventRecord(e[1], ids_s));
            if (!one_stream) FELOG_HIP(hipEventRecord(ready[set], ids_s));
        };
        const int64_t ahead = kIdSets - 1;
        for (int64_t k = 0; k < ahead && first_mb + k < end; ++k) issue_ids(first_mb + k);
        for (int64_t b = first_mb; b < end; ++b) {
            const int set = (int)(b % kIdSets);
            const MinibatchLaunch ml = mls[set];
            const float lr = lrs[set];
            hipEvent_t* e = slot_of[set];
            if (!one_stream) FELOG_HIP(hipStreamWaitEvent(c.stream, ready[set], 0));
            FwdArgs f = fa;
            f.lr = lr;
            f.npairs = ml.npairs;
            launch_train(m, m.mb[set], f, ml, meta0 + kMetaWords * set, nullptr, nullptr,
                         c.stream, e ? e + 2 : nullptr, one_stream ? nullptr : fwd_done);
            if (!one_stream) FELOG_HIP(hipEventRecord(freed[set], c.stream));
            pairs_done += ml.npairs;
            // later minibatches' ids run beside this one's apply launches and the
            // next forward, not beside this forward
            if (b + ahead < end) {
                if (!one_stream) FELOG_HIP(hipStreamWaitEvent(ids_s, fwd_done, 0));
                issue_ids(b + ahead);
            }
        }
    } else if (!apply) {
        // capture: the deltas of one minibatch, by touched-list position, not applied
        const int64_t b = first_mb;
        const int par = (int)(b % kIdSets);
        MinibatchLaunch ml;
        PrepArgs a = pa;
        const float lr = frame(b, ml, a);
        gate(c.stream, chunk);
        uint32_t* meta = meta0 + kMetaWords * par;
        DevBuf vin, vout;
        vin.alloc(&c, sizeof(float) * (size_t)P * m.dim);
        vout.alloc(&c, sizeof(float) * (size_t)P * (K + 1) * m.dim);
        FELOG_HIP(hipMemsetAsync(vin.ptr, 0, vin.bytes, c.stream));
        FELOG_HIP(hipMemsetAsync(vout.ptr, 0, vout.bytes, c.stream));
        launch_ids(m.mb[par], a, ml, meta, c.stream);
        FwdArgs f = fa;
        f.lr = lr;
        f.npairs = ml.npairs;
        launch_train(m, m.mb[par], f, ml, meta, vin.as<float>(), vout.as<float>(), c.stream,
                     nullptr);
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
        FELOG_HIP(hipMemcpyAsync(rows_in, m.mb[par].list_in.ptr, sizeof(int32_t) * ui,
                                 hipMemcpyDeviceToHost, c.stream));
        FELOG_HIP(hipMemcpyAsync(rows_out, m.mb[par].list_out.ptr, sizeof(int32_t) * uo,
                                 hipMemcpyDeviceToHost, c.stream));
        FELOG_HIP(hipMemcpyAsync(d_in_host, vin.ptr, sizeof(float) * ui * m.dim,
                                 hipMemcpyDeviceToHost, c.stream));
        FELOG_HIP(hipMemcpyAsync(d_out_host, vout.ptr, sizeof(float) * uo * m.dim,
                                 hipMemcpyDeviceToHost, c.stream));
        FELOG_HIP(hipMemsetAsync(m.row_totals.ptr, 0, sizeof(uint64_t) * 3, c.stream));
        c.sync();
        if (n_in) *n_in = ui;
        if (n_out) *n_out = uo;
        pairs_done += ml.npairs;
    }
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, c.stream,
                       loss_part.as<double>(), blocks * 4, m.loss_out.as<double>());
    FELOG_HIP(hipGetLastError());
    FELOG_HIP(hipEventRecord(c.ev1, c.stream));
    double loss = 0.0;
    unsigned long long rows[3] = {0, 0, 0};
    FELOG_HIP(hipMemcpyAsync(&loss, m.loss_out.ptr, sizeof loss, hipMemcpyDeviceToHost, c.stream));
    FELOG_HIP(hipMemcpyAsync(rows, m.row_totals.ptr, sizeof rows, hipMemcpyDeviceToHost,
                             c.stream));
    c.sync();
    if (c.aux) FELOG_HIP(hipStreamSynchronize(c.aux));
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
        stats->rows_out_single = (int64_t)rows[2];
        stats->timed_launches = timed;
        stats->ms_forward = ms_fwd;
        stats->ms_apply = ms_apply;
        stats->ms_apply_first = ms_apply_first;
        stats->ms_prep = ms_prep;
        stats->path = 0;
        stats->update_blocks = 0;
        stats->timed_minibatches = timed;
        stats->ms_update = 0.0;
    }
}

}  // namespace felog
