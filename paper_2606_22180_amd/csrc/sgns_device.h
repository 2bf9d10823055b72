// Device helpers shared by the SGNS update kernels (sgns.hip: per-minibatch
// launches; sgns_small.hip: the persistent small-minibatch update).
#pragma once

#include "common.h"

namespace felog {

// Stores with the nontemporal hint, for outputs the launch itself does not
// read again: the forward's per-touch outputs and the rows it and the apply
// launches write.  Measured on R-MAT 2^20 at 65,536 pairs: 153.6 -> 150.1 us
// per minibatch.  (On the split rows' partial sums, which the next launch
// reads, the hint made the minibatch slower.)
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef int nt_i2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_nt(float4* p, const float4& v)
{
    __builtin_nontemporal_store(nt_f4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_f4*>(p));
}
__device__ __forceinline__ void store_nt(int2* p, const int2& v)
{
    __builtin_nontemporal_store(nt_i2{v.x, v.y}, reinterpret_cast<nt_i2*>(p));
}
__device__ __forceinline__ void store_nt(uint32_t* p, uint32_t v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_nt(int4* p, const int4& v)
{
    typedef int nt_i4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(nt_i4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_i4*>(p));
}

constexpr int kChunk = 16;                // touches per reduction work item (one per lane of a group)
constexpr int kMetaWords = 16;            // per minibatch parity
// meta words (in, out): [0, 1] list lengths, [2, 3] rows of one chunk,
// [4, 5] rows split over chunks, [6, 7] chunks of split rows

// Adding c = 1.5 * 2^k rounds a value below 2^(k-1) in magnitude to a
// multiple of 2^(k-52); taking c off again is exact.
__device__ __forceinline__ double on_grid(double t, double c) { return __dsub_rn(__dadd_rn(t, c), c); }

__device__ __forceinline__ double wave_sum_f64(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// sigma(x) = 1 / (1 + exp(-x)) in FP64, without clipping (Eq. (2)).
__device__ __forceinline__ double sigmoid_d(double x) { return 1.0 / (1.0 + exp(-x)); }

// -log sigma(x) = log(1 + exp(-x)), without overflow.  A loss term is
// evaluated in FP32 from the FP64 dot (relative error ~1e-7 per term) and the
// terms are summed in FP64.
__device__ __forceinline__ float neg_log_sigmoid(float x)
{
    return fmaxf(-x, 0.0f) + log1pf(expf(-fabsf(x)));
}

__device__ __forceinline__ double dot4d(float4 a, float4 b, double acc)
{
    acc = fma((double)a.x, (double)b.x, acc);
    acc = fma((double)a.y, (double)b.y, acc);
    acc = fma((double)a.z, (double)b.z, acc);
    return fma((double)a.w, (double)b.w, acc);
}

// The FP64 coefficient g and the pair-order key of an out-touch, with the
// context row its delta draws on, in one 16-byte entry.
__device__ __forceinline__ int4 pack_entry(double g, int32_t ctx, uint32_t key)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(g);
    return make_int4((int32_t)(uint32_t)b, (int32_t)(uint32_t)(b >> 32), ctx, (int32_t)key);
}
__device__ __forceinline__ double entry_g(int4 e)
{
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)e.y << 32) |
                                            (uint32_t)e.x));
}

template <int D>
__device__ __forceinline__ const float4* row4(const float* base, int64_t row)
{
    return reinterpret_cast<const float4*>(base + row * D);
}

// The apply's row slots past a segment's end: zeros, with no load issued.
// Pointing those loads at row 0 instead made every short segment of the
// minibatch read the same line, which queued in one L2 channel (about 1 us
// per minibatch of the persistent update on R-MAT 2^20).
template <int D, int NV>
__device__ __forceinline__ void load_row_if(float4 (&x)[NV], const float* base, int32_t row,
                                            bool ok, int lane16)
{
#pragma unroll
    for (int i = 0; i < NV; ++i) x[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (ok) {
        const float4* r = row4<D>(base, row);
#pragma unroll
        for (int i = 0; i < NV; ++i) x[i] = r[i * 16 + lane16];
    }
}

__device__ __forceinline__ float dot4(float4 a, float4 b, float acc)
{
    acc = fmaf(a.x, b.x, acc);
    acc = fmaf(a.y, b.y, acc);
    acc = fmaf(a.z, b.z, acc);
    return fmaf(a.w, b.w, acc);
}

// Sum over the L lanes of a lane group (L = 16 or 32).
template <int L>
__device__ __forceinline__ float group_sum(float x)
{
    if (L > 16) x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 8);
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 1);
    return x;
}

// Lanes per pair in the forward: 16 at d = 64, 32 from d = 128.  With FP64
// dots and coefficients, 16 lanes at d = 128 needed 228 registers (two waves
// per SIMD); 32 lanes need 164 (three), and the forward at P = 65,536 on
// R-MAT 2^20 went from 103.9 to 91.9 us.
template <int D, int K>
constexpr int fwd_lanes_per_pair() { return D <= 64 ? 16 : 32; }

template <int L>
__device__ __forceinline__ double group_sum_d(double x);

// The pair's coefficients g[0..K] (Eq. (2) gradient weights, FP64):
// g0 = lr (1 - sigma(s0)), gk = -lr sigma(sk), 0 for a skipped negative,
// from FP64 dots over the group's LPP lanes.  Lane j of the group evaluates
// sigma and the loss term of touch j (and j + LPP), so each lane runs one
// FP64 exponential instead of K + 1; the coefficients are then broadcast.
// The loss term, -log sigma(s0) or -log sigma(-sk), is FP32 from the FP64
// dot, added to lacc in FP64.
template <int K, int LPP, int V4>
__device__ __forceinline__ void coefficients(const float4 (&vin)[V4], const float4 (&vo)[K + 1][V4],
                                             const int32_t (&t)[K + 1], double lr, bool live,
                                             int gl, int grp, double (&g)[K + 1], double& lacc)
{
    double dot[K + 1];
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < V4; ++i) acc = dot4d(vin[i], vo[k][i], acc);
        dot[k] = group_sum_d<LPP>(acc);
    }
    constexpr int H = (K + LPP) / LPP;   // touches per lane
    double mine[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int k = gl + h * LPP;
        double dk = dot[0];
        bool ok = true;
#pragma unroll
        for (int j = 1; j <= K; ++j)
            if (k == j) {
                dk = dot[j];
                ok = t[j] >= 0;
            }
        const double sg = sigmoid_d(dk);
        mine[h] = k == 0 ? lr * (1.0 - sg) : (ok ? -lr * sg : 0.0);
        if (k <= K && live && ok) lacc += (double)neg_log_sigmoid((float)(k == 0 ? dk : -dk));
    }
#pragma unroll
    for (int k = 0; k <= K; ++k) g[k] = __shfl(mine[k / LPP], grp * LPP + k % LPP);
}

template <int L>
__device__ __forceinline__ double group_sum_d(double x)
{
    if (L > 16) x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 8);
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 1);
    return x;
}

// The row's current values (zero when capturing), read before the delta is
// summed so that the read overlaps the summing.
template <int D>
__device__ __forceinline__ void get_row(const float* table, const float* cap, int32_t row,
                                        float4 (&cur)[D / 64], int gl)
{
    const float4* s4 = reinterpret_cast<const float4*>(table + (int64_t)row * D);
#pragma unroll
    for (int i = 0; i < D / 64; ++i) cur[i] = cap ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : s4[i * 16 + gl];
}

// Adds a row's FP64 delta to its current values (from get_row) and rounds
// once to FP32 into the table, or stores the delta rounded to FP32 in the
// capture buffer.
template <int D>
__device__ __forceinline__ void put_row(float* table, float* cap, int32_t row, int32_t slot,
                                        const float4 (&cur)[D / 64],
                                        const double (&delta)[D / 16], int gl)
{
    constexpr int V4 = D / 64;
    float4* d4 = reinterpret_cast<float4*>(cap ? cap + (int64_t)slot * D : table + (int64_t)row * D);
#pragma unroll
    for (int i = 0; i < V4; ++i) {
        const float4 c = cur[i];
        const float4 v = make_float4((float)((double)c.x + delta[4 * i + 0]),
                                     (float)((double)c.y + delta[4 * i + 1]),
                                     (float)((double)c.z + delta[4 * i + 2]),
                                     (float)((double)c.w + delta[4 * i + 3]));
        store_nt(&d4[i * 16 + gl], v);
    }
}

}  // namespace felog
