// Block-level scans and an order-preserving, deterministic compaction used by
// the walk, noise-distribution and feedback kernels.  256-thread blocks; each
// thread owns kItems consecutive items, so a block spans 2048 items.
#pragma once

#include "common.h"

namespace felog {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanSpan = kScanThreads * kScanItems;

// Exclusive scan of one value per thread across a 256-thread block.
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds /* [kScanThreads] */, T* total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    // Hillis-Steele inclusive scan in LDS (8 steps for 256 threads).
    for (int off = 1; off < kScanThreads; off <<= 1) {
        T add = t >= off ? lds[t - off] : T(0);
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    T incl = lds[t];
    if (total) *total = lds[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

// Pass 1: items kept per block.
template <class Pred>
__global__ __launch_bounds__(kScanThreads) void compact_count_kernel(Pred pred, int64_t n,
                                                                    uint32_t* block_counts)
{
    __shared__ uint32_t lds[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanSpan + (int64_t)threadIdx.x * kScanItems;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n && pred(base + k)) ++c;
    uint32_t total;
    block_exclusive_scan<uint32_t>(c, lds, &total);
    if (threadIdx.x == 0) block_counts[blockIdx.x] = total;
}

// Pass 2 (one block): exclusive scan of the per-block counts, total in out[nb].
static __global__ __launch_bounds__(kScanThreads) void scan_counts_kernel(uint32_t* counts, int64_t nb)
{
    __shared__ uint32_t lds[kScanThreads];
    uint32_t carry = 0;
    for (int64_t s = 0; s < nb; s += kScanThreads) {
        int64_t i = s + threadIdx.x;
        uint32_t v = i < nb ? counts[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<uint32_t>(v, lds, &tot);
        if (i < nb) counts[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) counts[nb] = carry;
}

// Pass 3: write kept values in item order.
template <class Pred, class Val>
__global__ __launch_bounds__(kScanThreads) void compact_scatter_kernel(
    Pred pred, Val val, int64_t n, const uint32_t* block_offsets, int32_t* out)
{
    __shared__ uint32_t lds[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanSpan + (int64_t)threadIdx.x * kScanItems;
    bool keep[kScanItems];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        keep[k] = base + k < n && pred(base + k);
        c += keep[k];
    }
    uint32_t pos = block_offsets[blockIdx.x] + block_exclusive_scan<uint32_t>(c, lds, nullptr);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (keep[k]) out[pos++] = val(base + k);
}

// Order-preserving compaction of val(i) for i in [0, n) with pred(i); returns
// the number kept (one 4-byte device-to-host copy).  `out` is (re)allocated.
template <class Pred, class Val>
int64_t compact(Ctx& ctx, Pred pred, Val val, int64_t n, DevBuf& out)
{
    int64_t nb = (n + kScanSpan - 1) / kScanSpan;
    DevBuf counts;
    counts.alloc(&ctx, sizeof(uint32_t) * (nb + 1));
    uint32_t* c = counts.as<uint32_t>();
    if (nb > 0) {
        hipLaunchKernelGGL(compact_count_kernel<Pred>, dim3(nb), dim3(kScanThreads), 0,
                           ctx.stream, pred, n, c);
        FELOG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(kScanThreads), 0, ctx.stream, c, nb);
    FELOG_HIP(hipGetLastError());
    uint32_t total = 0;
    FELOG_HIP(hipMemcpyAsync(&total, c + nb, sizeof total, hipMemcpyDeviceToHost, ctx.stream));
    ctx.sync();
    out.alloc(&ctx, sizeof(int32_t) * (total ? total : 1));
    if (total && nb > 0) {
        hipLaunchKernelGGL((compact_scatter_kernel<Pred, Val>), dim3(nb), dim3(kScanThreads), 0,
                           ctx.stream, pred, val, n, c, out.as<int32_t>());
        FELOG_HIP(hipGetLastError());
    }
    return total;
}

}  // namespace felog
