// Shared-negative SGNS on BF16 tables with MFMA (a systems form of Eq. (2);
// the paper trains in FP32 and does not describe it).
//
// A minibatch of P pairs (the same pair order as the FP32 path) shares M
// negatives.  With C = bf16 in[ctx] (P x d), O = bf16 out[ctr] (P x d) and
// N = bf16 out[neg] (M x d):
//   S  = C N^T                       (P x M, MFMA, FP32 accumulation)
//   G  = bf16(-lr (K/M) sigma(S) o mask),  mask = [neg != ctr] (and real pairs)
//   dC = G N,  dN = G^T C            (MFMA, FP32 accumulation)
//   g0 = lr (1 - sigma(C.O)) row-wise (FP32 dot of the BF16 rows)
//   in[ctx] += dC + g0 O,  out[neg] += dN,  out[ctr] += g0 C   on FP32 masters.
// The BF16 rows are the masters rounded to nearest even as they stand at the
// minibatch's start; the gather rounds them as it reads them, so no BF16
// copy of the tables has to be kept current.  Each (pair, negative) term
// weighs K/M, so the expected update equals Eq. (2) with K negatives per pair.
//
// Kernels per minibatch: gather (rows, transposed copies, positive terms),
// fused (S, G, dC and dN in one launch: a block takes a 16-row panel of one
// side and streams the other side in 32-row chunks, G passing from the score
// MFMAs to the output MFMAs in registers; each touch's FP32 term stored as a
// row of a delta buffer, in up to four parts), apply (one wave per touched
// row sums its touches' terms in FP64, in touch order, and adds the sum to
// the master with one rounding).  A row repeats when a node is the
// context of several pairs, the centre of several, a negative drawn twice, or
// both a centre and a negative; summing its terms in a fixed order instead of
// with atomics makes the tables bit-reproducible.  The touches' order comes
// from a plan that sorts them by (table, row, touch): in LDS, one workgroup
// per minibatch for up to 64 minibatches per launch, when 2P + M <= 8192,
// else a radix sort per minibatch (stable, so equal rows keep touch order).
// The ids (ctx, ctr, neg) of up to 64 minibatches come from one launch
// before them.
// MFMA: v_mfma_f32_16x16x32_bf16.  Lane l holds 8 consecutive k of row
// (l mod 16) of A and of column (l mod 16) of B, k chunk l / 16; it receives
// D[4 (l / 16) + j][l mod 16], j = 0..3.
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"
#include "noise.h"

namespace felog {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u) {                // inf / nan
        uint16_t h = (uint16_t)(u >> 16);
        if (u & 0x007FFFFFu) h |= 0x0040u;
        return h;
    }
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p)
{
    uint4 v = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(bf16x8, v);
}

struct Bf16Args {
    // tables
    float* tin;
    float* tout;
    int32_t d;
    // pair order (as the FP32 path)
    const int32_t* walks;
    int64_t W;
    const int32_t* vcols;
    uint32_t Wv;
    const int32_t* slices;
    uint32_t first_pair;
    uint32_t np;          // real pairs in this minibatch (<= P)
    int32_t window;
    // shared negatives
    uint32_t P, M;
    int32_t K;
    uint32_t mb;          // minibatch index b
    uint32_t id_lo;       // low 32 bits of the corpus's first walk id
    uint64_t seed;
    NoiseTable noise;
    float lr;
    // scratch
    int32_t* ids;         // ctx[P], ctr[P], neg[M]
    uint16_t* C;          // [P][d]
    uint16_t* O;          // [P][d]
    uint16_t* N;          // [M][d]
    uint16_t* Ct;         // [d][P]
    uint16_t* Nt;         // [d][M]
    float* g0;            // [P]
    double* loss_part;    // [P + M] gather slots, then one per pair block of the fused launch
    float* delta;         // [split][2P + M][d]: each touch's term (ctx, ctr, neg rows in
                          // touch order), as `split` partial sums over the shared dimension
    uint32_t split;       // blocks per panel of the fused launch (1, 2 or 4)
};

__device__ __forceinline__ float wave_sum32(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// log(1 + exp(x)) in FP32, without overflow; the loss sums these terms in FP64.
__device__ __forceinline__ float softplus_f(float x)
{
    return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}

// sigma(x) and log(1 + exp(-|x|)) from one hardware exp2, one reciprocal and
// one log2 (a few FP32 ulps; the fused launch rounds G to BF16 right after)
__device__ __forceinline__ void sigma_fast(float x, float& sig, float& l1p)
{
    const float e = __builtin_amdgcn_exp2f(-fabsf(x) * 1.4426950408889634f);
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    sig = x >= 0.0f ? r : e * r;
    l1p = __builtin_amdgcn_logf(1.0f + e) * 0.6931471805599453f;
}

// The ids of nmb consecutive minibatches of one chunk, mb0 first (their
// first pair is first0 within the chunk): for each, ctx[P] and ctr[P] (-1
// past the chunk's last pair) and neg[M], one thread per pair or negative.
// They read only the walks and the noise table, so one launch draws them for
// many minibatches and the per-minibatch launches start from the ids.
constexpr int kIdBatch = 64;

__global__ __launch_bounds__(256) void bf16_ids_kernel(Bf16Args a, uint32_t mb0, uint32_t nmb,
                                                       uint32_t first0, uint64_t chunk_pairs,
                                                       int32_t* ids)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t per = a.P + a.M;
    if (i >= (uint64_t)nmb * per) return;
    const uint32_t bm = (uint32_t)(i / per), s = (uint32_t)(i - (uint64_t)bm * per);
    int32_t* out = ids + (size_t)bm * (2 * a.P + a.M);
    if (s < a.P) {
        const uint64_t gq64 = (uint64_t)first0 + (uint64_t)bm * a.P + s;   // pair within the chunk
        int32_t ctx = -1, ctr = -1;
        if (gq64 < chunk_pairs) {
            const uint32_t gq = (uint32_t)gq64;
            const uint32_t sidx = gq / a.Wv;
            const uint32_t rank = gq - sidx * a.Wv;
            const int32_t js = a.slices[sidx];
            const int32_t col = a.vcols[rank];
            const int32_t j = js >> 8, sl = js & 255;
            const int32_t off = sl < a.window ? sl - a.window : sl - a.window + 1;
            ctx = a.walks[(int64_t)(j + off) * a.W + col];
            ctr = a.walks[(int64_t)j * a.W + col];
        }
        out[s] = ctx;
        out[a.P + s] = ctr;
    } else {
        const uint32_t m = s - a.P;
        Rand4 r = philox4x32(mb0 + bm, a.id_lo, m >> 1, kTagSharedNeg, a.seed);
        const uint32_t lo = (m & 1) ? r.v[2] : r.v[0];
        const uint32_t hi = (m & 1) ? r.v[3] : r.v[1];
        out[2 * a.P + m] = noise_draw(a.noise, ((uint64_t)hi << 32) | lo);
    }
}

// 16 rows per block, one per wave: blocks [0, P / 16) take pairs, the rest
// negatives (P and M are multiples of 64).  The rows are written as they are
// (C, O, N) and, through an LDS tile, transposed (C^T, N^T) as 16-byte runs
// of 8 consecutive rows.
constexpr int kGatherRows = 16;

template <int D>
__global__ __launch_bounds__(64 * kGatherRows) void bf16_gather_kernel(Bf16Args a)
{
    constexpr int RW = 1;                 // rows per wave
    constexpr int U = D / 64;             // elements per lane and row
    __shared__ __align__(16) uint16_t tile[D][kGatherRows + 8];   // [e][row of the block]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t r0 = blockIdx.x * kGatherRows;
    const bool pairs = r0 < a.P;
    if (pairs) {
        int32_t ctx[RW], ctr[RW];
        float xc[RW][U], xo[RW][U];
#pragma unroll
        for (int j = 0; j < RW; ++j) {
            const uint32_t p = r0 + wv * RW + j;
            ctx[j] = a.ids[p];
            ctr[j] = a.ids[a.P + p];
        }
#pragma unroll
        for (int j = 0; j < RW; ++j)        // all the row loads first
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + 64 * u;
                xc[j][u] = ctx[j] >= 0 ? a.tin[(int64_t)ctx[j] * D + e] : 0.0f;
                xo[j][u] = ctr[j] >= 0 ? a.tout[(int64_t)ctr[j] * D + e] : 0.0f;
            }
#pragma unroll
        for (int j = 0; j < RW; ++j) {
            const uint32_t p = r0 + wv * RW + j;
            float dot = 0.0f;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + 64 * u;
                const uint16_t c = ctx[j] >= 0 ? bf16_rne(xc[j][u]) : 0;
                const uint16_t o = ctr[j] >= 0 ? bf16_rne(xo[j][u]) : 0;
                a.C[(int64_t)p * D + e] = c;
                a.O[(int64_t)p * D + e] = o;
                tile[e][wv * RW + j] = c;
                dot = fmaf(bf16_to_f32(c), bf16_to_f32(o), dot);
            }
            dot = wave_sum32(dot);
            if (lane == 0) {
                float g = 0.0f;
                if (ctx[j] >= 0) {
                    g = a.lr * (1.0f - 1.0f / (1.0f + expf(-dot)));
                    a.loss_part[p] += (double)softplus_f(-dot);       // -log sigma(s0)
                }
                a.g0[p] = g;
            }
        }
    } else {
        int32_t neg[RW];
        float xn[RW][U];
#pragma unroll
        for (int j = 0; j < RW; ++j) neg[j] = a.ids[2 * a.P + (r0 - a.P) + wv * RW + j];
#pragma unroll
        for (int j = 0; j < RW; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) xn[j][u] = a.tout[(int64_t)neg[j] * D + lane + 64 * u];
#pragma unroll
        for (int j = 0; j < RW; ++j) {
            const uint32_t m = (r0 - a.P) + wv * RW + j;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = lane + 64 * u;
                const uint16_t x = bf16_rne(xn[j][u]);
                a.N[(int64_t)m * D + e] = x;
                tile[e][wv * RW + j] = x;
            }
        }
    }
    __syncthreads();
    uint16_t* T = pairs ? a.Ct : a.Nt;
    const uint32_t ld = pairs ? a.P : a.M;
    const uint32_t c0 = pairs ? r0 : r0 - a.P;
    for (int i = threadIdx.x; i < D * (kGatherRows / 8); i += blockDim.x) {
        const int e = i / (kGatherRows / 8), q = i % (kGatherRows / 8);
        *reinterpret_cast<uint4*>(T + (int64_t)e * ld + c0 + 8 * q) =
            *reinterpret_cast<const uint4*>(&tile[e][8 * q]);
    }
}

// Scores and gradients in one launch, G never stored.  A block owns a panel
// of 16 rows of one side and streams the other side in chunks of 32 rows:
//   panels [0, P/16):       panel = 16 pairs,      streamed = negatives,
//                           out = dC = G N  (16 x d)
//   panels [P/16, +M/16):   panel = 16 negatives,  streamed = pairs,
//                           out = dN = G^T C (16 x d)
// Each panel has `split` blocks (block = s * panels + panel), so that small
// minibatches still fill the chip; the chunks form 8 * split contiguous
// parts, and wave w of block s takes part (8 s + w + panel) mod 8 split, so
// that blocks of different panels read different chunks at a time.  Block s
// stores its partial sum as the touches' rows of delta part s; the apply
// adds the parts in order.
// Per chunk a wave computes the 32 x 16 score tile Y X^T (Y the streamed
// rows, X the panel) as two 16x16 MFMA tiles, so that lane l holds the
// scores of panel row l mod 16 against streamed rows 4 (l / 16) + j and
// 16 + 4 (l / 16) + j (j < 4).  Those 8 G values are exactly an A operand of
// the output contraction for panel row l mod 16 if the contraction's k index
// runs over the chunk's streamed rows in that order (any order of k gives
// the same sum's terms); the B operand takes the same rows from the
// transposed copy Y^T.  So G goes from the score accumulators to the next
// MFMA in registers.  The waves' partial outputs meet in LDS and are added
// in wave order; every element's terms are then stored as the touches'
// rows of the delta buffer: dC + g0 O and g0 C for a pair, dN for a negative.
// Pair blocks also sum the negative loss terms, one slot per block.
constexpr int kFusedWaves = 8;

template <int D>
__global__ __launch_bounds__(64 * kFusedWaves) void bf16_fused_kernel(Bf16Args a)
{
    constexpr int KS = D / 32;   // k steps of a score tile
    constexpr int ET = D / 16;   // 16-wide output tiles
    __shared__ float part[kFusedWaves][16][D + 4];
    __shared__ double lred[kFusedWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, q = lane >> 4;
    const uint32_t npb = a.P / 16;
    const uint32_t panels = npb + a.M / 16;
    const uint32_t sp = blockIdx.x / panels, panel = blockIdx.x - sp * panels;
    const bool isC = panel < npb;
    const uint32_t x0 = (isC ? panel : panel - npb) * 16;
    const uint16_t* X = isC ? a.C : a.N;
    const uint16_t* Y = isC ? a.N : a.C;
    const uint16_t* Yt = isC ? a.Nt : a.Ct;
    const uint32_t ny = isC ? a.M : a.P;
    // ids: a pair's centre (-1 past the chunk's end), a negative's node; a
    // term is kept when both are real and differ
    const int32_t* yid = isC ? a.ids + 2 * a.P : a.ids + a.P;
    const int32_t pv = isC ? a.ids[a.P + x0 + li] : a.ids[2 * a.P + x0 + li];
    bf16x8 xf[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) xf[s] = load8(X + (int64_t)(x0 + li) * D + 32 * s + 8 * q);
    f32x4 acc[ET];
#pragma unroll
    for (int t = 0; t < ET; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const float wk = -a.lr * (float)a.K / (float)a.M;
    const double lw = (double)a.K / (double)a.M;
    double lacc = 0.0;
    const uint32_t chunks = ny / 32;
    const uint32_t nparts = kFusedWaves * a.split;
    const uint32_t part_id = (sp * kFusedWaves + wv + panel) % nparts;
    const uint32_t c0 = (uint32_t)((uint64_t)chunks * part_id / nparts);
    const uint32_t c1 = (uint32_t)((uint64_t)chunks * (part_id + 1) / nparts);
    for (uint32_t ch = c0; ch < c1; ++ch) {
        const uint32_t y0 = ch * 32;
        bf16x8 yf[2][KS];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int s = 0; s < KS; ++s)
                yf[h][s] = load8(Y + (int64_t)(y0 + 16 * h + li) * D + 32 * s + 8 * q);
        int4 ids2[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
            ids2[h] = *reinterpret_cast<const int4*>(yid + y0 + 16 * h + 4 * q);
        f32x4 sc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            sc[h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < KS; ++s)
                sc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yf[h][s], xf[s], sc[h], 0, 0, 0);
        }
        uint32_t gw[4];   // G as 8 BF16 values, streamed rows 4q + j then 16 + 4q + j
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t iv[4] = {ids2[h].x, ids2[h].y, ids2[h].z, ids2[h].w};
            uint32_t gb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float x = sc[h][j];
                const int32_t sv = iv[j];
                float g = 0.0f;
                if (pv >= 0 && sv >= 0 && pv != sv) {
                    float sig, l1p;
                    sigma_fast(x, sig, l1p);
                    g = wk * sig;
                    // -(K/M) log sigma(-s) = (K/M) (max(s, 0) + log(1 + exp(-|s|)))
                    if (isC) lacc += lw * (double)(fmaxf(x, 0.0f) + l1p);
                }
                gb[j] = bf16_rne(g);
            }
            gw[2 * h] = gb[0] | (gb[1] << 16);
            gw[2 * h + 1] = gb[2] | (gb[3] << 16);
        }
        const bf16x8 ga = __builtin_bit_cast(bf16x8, make_uint4(gw[0], gw[1], gw[2], gw[3]));
        // B operands of the output contraction, loaded after the scores: with
        // them in flight beside the score operands the kernel needs more than
        // 128 VGPRs, which halves the resident blocks (measured slower)
#pragma unroll
        for (int t = 0; t < ET; ++t) {
            uint2 bt[2];
#pragma unroll
            for (int h = 0; h < 2; ++h)
                bt[h] = *reinterpret_cast<const uint2*>(Yt + (int64_t)(16 * t + li) * ny + y0 +
                                                        16 * h + 4 * q);
            const bf16x8 b =
                __builtin_bit_cast(bf16x8, make_uint4(bt[0].x, bt[0].y, bt[1].x, bt[1].y));
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ga, b, acc[t], 0, 0, 0);
        }
    }
    // acc[t][j] is element (4q + j, 16 t + li) of the block's 16 x D output
#pragma unroll
    for (int t = 0; t < ET; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[wv][4 * q + j][16 * t + li] = acc[t][j];
    if (isC) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lacc += __shfl_xor(lacc, off);
        if (lane == 0) lred[wv] = lacc;
    }
    __syncthreads();
    if (isC && threadIdx.x == 0) {
        double l = 0.0;
        for (int w = 0; w < kFusedWaves; ++w) l += lred[w];
        a.loss_part[a.P + a.M + sp * npb + panel] += l;
    }
    float* const dpart = a.delta + (size_t)sp * (2 * a.P + a.M) * D;
    for (int i = threadIdx.x; i < 16 * D; i += 64 * kFusedWaves) {
        const int row = i / D, e = i % D;
        float v = part[0][row][e];
#pragma unroll
        for (int w = 1; w < kFusedWaves; ++w) v += part[w][row][e];
        const uint32_t r = x0 + row;
        if (isC) {
            if (a.ids[r] < 0) continue;          // no pair in this row
            if (sp == 0) {                       // the positive terms go with part 0
                const float g = a.g0[r];
                const float o = bf16_to_f32(a.O[(int64_t)r * D + e]);
                const float c = bf16_to_f32(a.C[(int64_t)r * D + e]);
                dpart[(int64_t)r * D + e] = v + g * o;
                dpart[(int64_t)(a.P + r) * D + e] = g * c;
            } else {
                dpart[(int64_t)r * D + e] = v;
            }
        } else {
            dpart[(int64_t)(2 * a.P + r) * D + e] = v;
        }
    }
}

// ------------------------------------------------------------------ apply
// Touch t of a minibatch: t < P the context of pair t (in table), P <= t < 2P
// the centre of pair t - P, 2P <= t the negative t - 2P (out table).  Its
// sort key is (table << rb) | row with n < 2^rb; a pair past the chunk's end
// has key (2 << rb) - 1, which sorts after every real touch.
__device__ __forceinline__ uint32_t touch_key(int32_t row, uint32_t t, uint32_t P, uint32_t rb)
{
    if (row < 0) return (uint32_t)((2ull << rb) - 1);
    return ((t >= P ? 1u : 0u) << rb) | (uint32_t)row;
}

// Plan of up to 64 minibatches with 2P + M <= kBfPlanMax, one workgroup per
// minibatch: keys (key << 16 | t) in LDS, bitonic sort ascending, then the
// sorted keys and touches.
constexpr int kBfPlanThreads = 512;
constexpr uint32_t kBfPlanMax = 8192;

__global__ __launch_bounds__(kBfPlanThreads) void bf16_plan_kernel(const int32_t* ids, uint32_t P,
                                                                   uint32_t M, uint32_t rb,
                                                                   uint32_t* skey, uint32_t* stouch)
{
    __shared__ unsigned long long keys[kBfPlanMax];
    const uint32_t nt = 2 * P + M;
    uint32_t N = 64;
    while (N < nt) N <<= 1;
    const int32_t* id = ids + (size_t)blockIdx.x * nt;
    for (uint32_t t = threadIdx.x; t < N; t += kBfPlanThreads)
        keys[t] = t < nt ? ((unsigned long long)touch_key(id[t], t, P, rb) << 16) | t : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= N; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < N; i += kBfPlanThreads) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const unsigned long long x = keys[i], y = keys[l];
                    if ((x > y) == ((i & k) == 0)) {
                        keys[i] = y;
                        keys[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    uint32_t* sk = skey + (size_t)blockIdx.x * nt;
    uint32_t* st = stouch + (size_t)blockIdx.x * nt;
    for (uint32_t i = threadIdx.x; i < nt; i += kBfPlanThreads) {
        const unsigned long long x = keys[i];
        sk[i] = (uint32_t)(x >> 16);
        st[i] = (uint32_t)(x & 0xFFFF);
    }
}

// Sort input of one large minibatch: key and touch per touch.
__global__ void bf16_keys_kernel(const int32_t* ids, uint32_t P, uint32_t M, uint32_t rb,
                                 uint32_t* kin, uint32_t* vin)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * P + M) return;
    kin[t] = touch_key(ids[t], t, P, rb);
    vin[t] = t;
}

// One wave per sorted position; the wave at the first position of a row sums
// the terms of the row's touches in FP64, in sorted (touch) order and part
// order within a touch (a centre's term has part 0 only), 64 keys at a time,
// and adds the sum to the row with one rounding.
template <int D>
__global__ __launch_bounds__(256) void bf16_apply_kernel(const uint32_t* skey,
                                                         const uint32_t* stouch, uint32_t nt,
                                                         uint32_t rb, uint32_t P, uint32_t split,
                                                         const float* delta, float* tin,
                                                         float* tout)
{
    constexpr int U = D / 64;
    const int lane = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nt) return;
    const uint32_t key = skey[i];
    if (key == (uint32_t)((2ull << rb) - 1) || (i > 0 && skey[i - 1] == key)) return;
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    for (uint32_t j0 = i;; j0 += 64) {
        const uint32_t j = j0 + lane;
        const bool same = j < nt && skey[j] == key;
        const unsigned long long ends = __ballot(!same);
        const int len = ends ? __ffsll((long long)ends) - 1 : 64;
        const uint32_t mine = same ? stouch[j] : 0u;
#pragma unroll 4
        for (int q = 0; q < len; ++q) {
            const uint32_t t = __shfl(mine, q);
            const uint32_t parts = (t >= P && t < 2 * P) ? 1u : split;
            for (uint32_t s = 0; s < parts; ++s) {
                const float* row = delta + ((size_t)s * nt + t) * D;
#pragma unroll
                for (int u = 0; u < U; ++u) acc[u] += (double)row[lane + 64 * u];
            }
        }
        if (len < 64) break;
    }
    const uint32_t row = key & ((1u << rb) - 1);
    float* T = (key >> rb) ? tout : tin;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        float* x = T + (int64_t)row * D + lane + 64 * u;
        *x = (float)((double)*x + acc[u]);
    }
}

__global__ void bf16_from_master_kernel(const float* src, uint16_t* dst, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = bf16_rne(src[i]);
}

void bf16_refresh_all(Model& m)
{
    if (m.precision != FELOG_PREC_BF16) return;
    Ctx& c = *m.ctx;
    const int64_t count = (int64_t)m.g->n * m.dim;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(bf16_from_master_kernel, dim3(blocks), dim3(256), 0, c.stream,
                       m.tin.as<float>(), m.bin.as<uint16_t>(), count);
    hipLaunchKernelGGL(bf16_from_master_kernel, dim3(blocks), dim3(256), 0, c.stream,
                       m.tout.as<float>(), m.bout.as<uint16_t>(), count);
    FELOG_HIP(hipGetLastError());
}

__global__ void loss_sum_kernel(const double* part, int64_t n, double* out)
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

void train_minibatches_bf16(Model& m, Walks& w, const felog_train_params& p,
                            const TrainSchedule& sch, const int32_t* d_slices, int64_t first_mb,
                            int64_t end, float* cap_in, float* cap_out, felog_train_stats* stats)
{
    Ctx& c = *m.ctx;
    const uint32_t P = (uint32_t)p.minibatch_pairs, M = (uint32_t)p.shared_negatives;
    const uint32_t nt = 2 * P + M;               // touches per minibatch
    const bool lds_plan = nt <= kBfPlanMax;
    const int d = m.dim;
    uint32_t rb = 1;
    while (((int64_t)1 << rb) <= m.g->n) ++rb;   // n < 2^rb
    if (m.bf_P < P || m.bf_M < M) {
        m.bf_P = std::max(m.bf_P, P);
        m.bf_M = std::max(m.bf_M, M);
        const size_t cp = m.bf_P, cm = m.bf_M, ct = 2 * cp + cm;
        m.bf_ids.alloc(&c, sizeof(int32_t) * ct * kIdBatch);
        m.bf_C.alloc(&c, sizeof(uint16_t) * cp * d);
        m.bf_O.alloc(&c, sizeof(uint16_t) * cp * d);
        m.bf_N.alloc(&c, sizeof(uint16_t) * cm * d);
        m.bf_Ct.alloc(&c, sizeof(uint16_t) * cp * d);
        m.bf_Nt.alloc(&c, sizeof(uint16_t) * cm * d);
        m.bf_g0.alloc(&c, sizeof(float) * cp);
        // a launch group's LDS plans or one large minibatch's sorted touches
        const size_t sorted = std::max(ct, (size_t)kIdBatch * std::min<size_t>(ct, kBfPlanMax));
        m.bf_skey.alloc(&c, sizeof(uint32_t) * sorted);
        m.bf_stouch.alloc(&c, sizeof(uint32_t) * sorted);
        m.bf_kin.release();
        m.bf_vin.release();
        m.bf_sort_tmp.release();
    }
    // blocks per panel of the fused launch: at least 512 blocks where 4 suffice
    const uint32_t panels = P / 16 + M / 16;
    uint32_t split = 1;
    while (split < 4 && panels * split < 512) split *= 2;
    if (m.bf_delta.bytes < sizeof(float) * split * (size_t)nt * d)
        m.bf_delta.alloc(&c, sizeof(float) * split * (size_t)nt * d);
    if (!lds_plan && !m.bf_sort_tmp.ptr) {
        const size_t ct = 2 * (size_t)m.bf_P + m.bf_M;
        m.bf_kin.alloc(&c, sizeof(uint32_t) * ct);
        m.bf_vin.alloc(&c, sizeof(uint32_t) * ct);
        size_t tmp = 0;
        FELOG_HIP(rocprim::radix_sort_pairs(nullptr, tmp, (const uint32_t*)nullptr,
                                            (uint32_t*)nullptr, (const uint32_t*)nullptr,
                                            (uint32_t*)nullptr, (uint32_t)ct, 0u, 32u, c.stream));
        m.bf_sort_tmp.alloc(&c, std::max<size_t>(tmp, 256));
    }
    const int64_t nslots = (int64_t)P + M + (int64_t)split * (P / 16);
    DevBuf loss_part;
    loss_part.alloc(&c, sizeof(double) * nslots);
    FELOG_HIP(hipMemsetAsync(loss_part.ptr, 0, sizeof(double) * nslots, c.stream));

    Bf16Args a{};
    a.tin = m.tin.as<float>();
    a.tout = m.tout.as<float>();
    a.d = d;
    a.walks = w.data.as<int32_t>();
    a.W = w.W;
    a.slices = d_slices;
    a.window = p.window;
    a.P = P;
    a.M = M;
    a.K = p.negatives;
    a.id_lo = (uint32_t)w.id_base;
    a.seed = p.seed;
    a.noise = NoiseTable{m.cdf.as<uint64_t>(), m.guide.as<int32_t>(), m.total_weight, m.guide_bits};
    a.ids = m.bf_ids.as<int32_t>();
    a.C = m.bf_C.as<uint16_t>();
    a.O = m.bf_O.as<uint16_t>();
    a.N = m.bf_N.as<uint16_t>();
    a.Ct = m.bf_Ct.as<uint16_t>();
    a.Nt = m.bf_Nt.as<uint16_t>();
    a.g0 = m.bf_g0.as<float>();
    a.loss_part = loss_part.as<double>();
    a.delta = m.bf_delta.as<float>();
    a.split = split;
    // capture: the sums go to dense zeroed tables instead of the masters
    float* const dst_in = cap_in ? cap_in : m.tin.as<float>();
    float* const dst_out = cap_out ? cap_out : m.tout.as<float>();

    const double lr0 = (double)p.lr_start, lr1 = (double)p.lr_end;
    const uint32_t row_blocks = (P + M) / kGatherRows;
    const uint32_t fused_blocks = panels * split;
    int64_t pairs_done = 0;
    FELOG_HIP(hipEventRecord(c.ev0, c.stream));
    size_t chunk = 0;
    size_t gated = 0;   // walk chunks [0, gated) are known to be written
    int32_t* const ids0 = m.bf_ids.as<int32_t>();
    uint32_t* const skey0 = m.bf_skey.as<uint32_t>();
    uint32_t* const stouch0 = m.bf_stouch.as<uint32_t>();
    int64_t batch0 = first_mb, batch_end = first_mb;   // minibatches whose ids are drawn
    for (int64_t b = first_mb; b < end; ++b) {
        while (chunk + 1 < sch.chunk_first_mb.size() && sch.chunk_first_mb[chunk + 1] <= b) ++chunk;
        const int64_t local = b - sch.chunk_first_mb[chunk];
        const int64_t first = local * (int64_t)P;
        const int64_t np = std::min<int64_t>(P, sch.chunk_pairs[chunk] - first);
        a.vcols = w.valid_cols.as<int32_t>() + sch.chunk_valid_base[chunk];
        a.Wv = (uint32_t)w.chunk_valid[chunk];
        a.first_pair = (uint32_t)first;
        a.np = (uint32_t)np;
        a.mb = (uint32_t)b;
        if (b == batch_end) {
            // ids (and, when they fit in LDS, plans) of the next minibatches,
            // up to kIdBatch and the chunk's end
            while (gated <= chunk && gated < w.chunk_ready.size())
                FELOG_HIP(hipStreamWaitEvent(c.stream, w.chunk_ready[gated++], 0));
            int64_t lim = std::min<int64_t>(end, b + kIdBatch);
            if (chunk + 1 < sch.chunk_first_mb.size())
                lim = std::min<int64_t>(lim, sch.chunk_first_mb[chunk + 1]);
            batch0 = b;
            batch_end = lim;
            const uint64_t items = (uint64_t)(lim - b) * (P + M);
            hipLaunchKernelGGL(bf16_ids_kernel, dim3((uint32_t)((items + 255) / 256)), dim3(256),
                               0, c.stream, a, (uint32_t)b, (uint32_t)(lim - b), (uint32_t)first,
                               (uint64_t)sch.chunk_pairs[chunk], ids0);
            if (lds_plan)
                hipLaunchKernelGGL(bf16_plan_kernel, dim3((uint32_t)(lim - b)),
                                   dim3(kBfPlanThreads), 0, c.stream, ids0, P, M, rb, skey0,
                                   stouch0);
        }
        a.ids = ids0 + (size_t)(b - batch0) * nt;
        const uint32_t* skey = skey0;
        const uint32_t* stouch = stouch0;
        if (lds_plan) {
            skey += (size_t)(b - batch0) * nt;
            stouch += (size_t)(b - batch0) * nt;
        } else {
            hipLaunchKernelGGL(bf16_keys_kernel, dim3((nt + 255) / 256), dim3(256), 0, c.stream,
                               a.ids, P, M, rb, m.bf_kin.as<uint32_t>(), m.bf_vin.as<uint32_t>());
            size_t tmp = m.bf_sort_tmp.bytes;
            FELOG_HIP(rocprim::radix_sort_pairs(m.bf_sort_tmp.ptr, tmp,
                                                (const uint32_t*)m.bf_kin.as<uint32_t>(), skey0,
                                                (const uint32_t*)m.bf_vin.as<uint32_t>(), stouch0,
                                                nt, 0u, rb + 1, c.stream));
        }
        a.lr = (float)(lr0 - (lr0 - lr1) * (double)b / (double)std::max<int64_t>(1, sch.B - 1));
        const dim3 agrid((nt + 3) / 4);
        const dim3 fgrid(fused_blocks), fblock(64 * kFusedWaves);
        if (d == 64) {
            hipLaunchKernelGGL(bf16_gather_kernel<64>, dim3(row_blocks), dim3(64 * kGatherRows), 0, c.stream, a);
            hipLaunchKernelGGL(bf16_fused_kernel<64>, fgrid, fblock, 0, c.stream, a);
        } else if (d == 128) {
            hipLaunchKernelGGL(bf16_gather_kernel<128>, dim3(row_blocks), dim3(64 * kGatherRows), 0, c.stream, a);
            hipLaunchKernelGGL(bf16_fused_kernel<128>, fgrid, fblock, 0, c.stream, a);
        } else {
            hipLaunchKernelGGL(bf16_gather_kernel<256>, dim3(row_blocks), dim3(64 * kGatherRows), 0, c.stream, a);
            hipLaunchKernelGGL(bf16_fused_kernel<256>, fgrid, fblock, 0, c.stream, a);
        }
        if (d == 64)
            hipLaunchKernelGGL(bf16_apply_kernel<64>, agrid, dim3(256), 0, c.stream, skey, stouch,
                               nt, rb, P, split, (const float*)a.delta, dst_in, dst_out);
        else if (d == 128)
            hipLaunchKernelGGL(bf16_apply_kernel<128>, agrid, dim3(256), 0, c.stream, skey, stouch,
                               nt, rb, P, split, (const float*)a.delta, dst_in, dst_out);
        else
            hipLaunchKernelGGL(bf16_apply_kernel<256>, agrid, dim3(256), 0, c.stream, skey, stouch,
                               nt, rb, P, split, (const float*)a.delta, dst_in, dst_out);
        FELOG_HIP(hipGetLastError());
        pairs_done += np;
    }
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, c.stream, loss_part.as<double>(),
                       nslots, m.loss_out.as<double>());
    FELOG_HIP(hipGetLastError());
    FELOG_HIP(hipEventRecord(c.ev1, c.stream));
    double loss = 0.0;
    FELOG_HIP(hipMemcpyAsync(&loss, m.loss_out.ptr, sizeof loss, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    float ms = 0.0f;
    FELOG_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    if (stats) {
        *stats = felog_train_stats{};
        stats->minibatches = end - first_mb;
        stats->pairs = pairs_done;
        stats->minibatches_total = sch.B;
        stats->loss = loss;
        stats->ms = ms;
    }
}

}  // namespace felog
