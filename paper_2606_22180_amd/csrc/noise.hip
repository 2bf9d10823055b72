// Embedding initialisation and the negative-sampling noise distribution
// Pn(u) of Eq. (2).
//
// Pn(u) ~ c_u^0.75, where c is a node's degree or its occurrence count in a
// walk corpus.  Weights are integers, W_u = floor(2^16 * sqrt(c) * sqrt(sqrt(c)))
// in IEEE double (sqrt and multiply correctly rounded), so the cumulative
// weights are exact and a draw is the exact inverse CDF of a 64-bit uniform:
// u = floor(x * T / 2^64), answer = the node whose interval [cdf[i], cdf[i+1])
// holds u.  A guide table (Chen & Asau's indexed search) over the top bits of
// x gives a starting node no larger than the answer, from which a short
// forward scan finds it: O(1) expected reads per draw.
#include "common.h"
#include "noise.h"

namespace felog {

// in[v][c] = ((x >> 8) * 2^-24 - 0.5) / d, x = word c mod 4 of Philox(v, c/4, 0, INIT).
__global__ void init_tables_kernel(float* __restrict__ tin, int32_t n, int32_t d, uint64_t seed)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one thread per 4 entries
    int64_t quads = (int64_t)n * (d / 4);
    if (i >= quads) return;
    int64_t v = i / (d / 4);
    uint32_t c4 = (uint32_t)(i - v * (d / 4));
    Rand4 r = philox4x32((uint32_t)v, (uint32_t)(v >> 32), c4, kTagInit, seed);
    float4 o;
    const float inv = 1.0f / 16777216.0f;
    o.x = ((float)(r.v[0] >> 8) * inv - 0.5f) / (float)d;
    o.y = ((float)(r.v[1] >> 8) * inv - 0.5f) / (float)d;
    o.z = ((float)(r.v[2] >> 8) * inv - 0.5f) / (float)d;
    o.w = ((float)(r.v[3] >> 8) * inv - 0.5f) / (float)d;
    reinterpret_cast<float4*>(tin)[i] = o;
}

void launch_init_tables(Model& m, uint64_t seed)
{
    Ctx& c = *m.ctx;
    int64_t quads = (int64_t)m.g->n * (m.dim / 4);
    hipLaunchKernelGGL(init_tables_kernel, dim3((quads + 255) / 256), dim3(256), 0, c.stream,
                       m.tin.as<float>(), m.g->n, m.dim, seed);
    FELOG_HIP(hipGetLastError());
    FELOG_HIP(hipMemsetAsync(m.tout.ptr, 0, sizeof(float) * (size_t)m.g->n * m.dim, c.stream));
}

__global__ void degree_counts_kernel(const int64_t* indptr, int32_t n, uint32_t* counts)
{
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) counts[v] = (uint32_t)(indptr[v + 1] - indptr[v]);
}

void launch_degree_counts(Graph& g, uint32_t* d_counts)
{
    Ctx& c = *g.ctx;
    hipLaunchKernelGGL(degree_counts_kernel, dim3((g.n + 255) / 256), dim3(256), 0, c.stream,
                       g.indptr.as<int64_t>(), g.n, d_counts);
    FELOG_HIP(hipGetLastError());
}

// Occurrences of each node in a walk corpus (integer atomics: order-free).
__global__ void corpus_counts_kernel(const int32_t* __restrict__ walks, int64_t total,
                                     uint32_t* counts)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        int32_t v = walks[i];
        if (v >= 0) atomicAdd(&counts[v], 1u);
    }
}

void launch_corpus_counts(const Walks& w, uint32_t* d_counts)
{
    Ctx& c = *w.g->ctx;
    FELOG_HIP(hipMemsetAsync(d_counts, 0, sizeof(uint32_t) * w.g->n, c.stream));
    int64_t total = w.W * w.L;
    if (total == 0) return;
    int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(corpus_counts_kernel, dim3(blocks), dim3(256), 0, c.stream,
                       w.data.as<int32_t>(), total, d_counts);
    FELOG_HIP(hipGetLastError());
}

// W_u = floor(2^16 * sqrt(c) * sqrt(sqrt(c))).
__global__ void noise_weights_kernel(const uint32_t* counts, int32_t n, uint64_t* w)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double c = (double)counts[i];
    double s = __dsqrt_rn(c);
    double t = __dsqrt_rn(s);
    double x = __dmul_rn(s, t);
    w[i] = (uint64_t)__dmul_rn(x, 65536.0);
}

// Inclusive scan of 64-bit weights into cdf[1..n] (cdf[0] = 0), three passes.
__global__ __launch_bounds__(256) void block_sums_u64(const uint64_t* w, int32_t n,
                                                      uint64_t* sums)
{
    __shared__ uint64_t lds[256];
    int64_t base = (int64_t)blockIdx.x * 2048 + threadIdx.x * 8;
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (base + k < n) acc += w[base + k];
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = lds[0];
}

__global__ __launch_bounds__(256) void scan_sums_u64(uint64_t* sums, int64_t nb)
{
    // one block: exclusive scan in place, total written to sums[nb]
    __shared__ uint64_t lds[256];
    uint64_t carry = 0;
    for (int64_t s = 0; s < nb; s += 256) {
        int64_t i = s + threadIdx.x;
        uint64_t v = i < nb ? sums[i] : 0;
        lds[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            uint64_t add = threadIdx.x >= off ? lds[threadIdx.x - off] : 0;
            __syncthreads();
            lds[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + lds[threadIdx.x] - v;
        uint64_t tot = lds[255];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(256) void finish_cdf_u64(const uint64_t* w, int32_t n,
                                                      const uint64_t* offsets, uint64_t* cdf)
{
    __shared__ uint64_t lds[256];
    int64_t base = (int64_t)blockIdx.x * 2048 + threadIdx.x * 8;
    uint64_t vals[8];
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        vals[k] = base + k < n ? w[base + k] : 0;
        acc += vals[k];
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint64_t add = threadIdx.x >= off ? lds[threadIdx.x - off] : 0;
        __syncthreads();
        lds[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t run = offsets[blockIdx.x] + lds[threadIdx.x] - acc;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (base + k < n) {
            run += vals[k];
            cdf[base + k + 1] = run;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) cdf[0] = 0;
}

// guide[b] = first node whose interval reaches past the smallest u of bucket b.
__global__ void guide_kernel(const uint64_t* cdf, int32_t n, int32_t bits, uint64_t total,
                             int32_t* guide)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= (int64_t)1 << bits) return;
    uint64_t x = (uint64_t)b << (64 - bits);
    uint64_t u = __umul64hi(x, total);
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
    }
    guide[b] = lo;
}

// guide table of m.cdf (n + 1 entries, total > 0)
static void build_guide(Model& m, uint64_t total)
{
    Ctx& c = *m.ctx;
    const int32_t n = m.g->n;
    int32_t bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < n) ++bits;
    m.guide_bits = bits;
    m.total_weight = total;
    m.guide.alloc(&c, sizeof(int32_t) * ((size_t)1 << bits));
    hipLaunchKernelGGL(guide_kernel, dim3((((int64_t)1 << bits) + 255) / 256), dim3(256), 0,
                       c.stream, m.cdf.as<uint64_t>(), n, bits, total, m.guide.as<int32_t>());
    FELOG_HIP(hipGetLastError());
    c.sync();
    m.have_noise = true;
}

void set_noise_cdf(Model& m, const uint64_t* host_cdf)
{
    Ctx& c = *m.ctx;
    const int32_t n = m.g->n;
    FELOG_REQUIRE(host_cdf[0] == 0, "a noise table starts at 0");
    for (int32_t i = 0; i < n; ++i)
        FELOG_REQUIRE(host_cdf[i + 1] >= host_cdf[i], "the noise table decreases at node %d", i);
    FELOG_REQUIRE(host_cdf[n] > 0, "the noise distribution is empty (every weight is zero)");
    m.cdf.alloc(&c, sizeof(uint64_t) * (n + 1));
    FELOG_HIP(hipMemcpyAsync(m.cdf.ptr, host_cdf, sizeof(uint64_t) * (n + 1),
                             hipMemcpyHostToDevice, c.stream));
    build_guide(m, host_cdf[n]);
}

void build_noise_from_counts(Model& m, const uint32_t* d_counts)
{
    Ctx& c = *m.ctx;
    int32_t n = m.g->n;
    DevBuf w;
    w.alloc(&c, sizeof(uint64_t) * n);
    hipLaunchKernelGGL(noise_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, c.stream,
                       d_counts, n, w.as<uint64_t>());
    FELOG_HIP(hipGetLastError());
    int64_t nb = (n + 2047) / 2048;
    DevBuf sums;
    sums.alloc(&c, sizeof(uint64_t) * (nb + 1));
    m.cdf.alloc(&c, sizeof(uint64_t) * (n + 1));
    hipLaunchKernelGGL(block_sums_u64, dim3(nb), dim3(256), 0, c.stream, w.as<uint64_t>(), n,
                       sums.as<uint64_t>());
    hipLaunchKernelGGL(scan_sums_u64, dim3(1), dim3(256), 0, c.stream, sums.as<uint64_t>(), nb);
    hipLaunchKernelGGL(finish_cdf_u64, dim3(nb), dim3(256), 0, c.stream, w.as<uint64_t>(), n,
                       sums.as<uint64_t>(), m.cdf.as<uint64_t>());
    FELOG_HIP(hipGetLastError());
    uint64_t total = 0;
    FELOG_HIP(hipMemcpyAsync(&total, m.cdf.as<uint64_t>() + n, sizeof total,
                             hipMemcpyDeviceToHost, c.stream));
    c.sync();
    FELOG_REQUIRE(total > 0, "the noise distribution is empty (every count is zero)");
    build_guide(m, total);
}

}  // namespace felog
