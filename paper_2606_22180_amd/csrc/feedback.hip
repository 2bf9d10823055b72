// Feedback of FeeST (Section 5.1): Psi of Eq. (4) and the next active set of
// Eq. (5).
//
// Psi(v) is the mean cosine similarity between v's input embedding and those
// of a neighbour subset: every neighbour when deg(v) <= k_s, otherwise k_s
// distinct neighbours chosen by Floyd's algorithm (Bentley & Floyd, 1987),
// draw m from word m mod 4 of Philox(v, round, m / 4, PSI).  Products and sums
// are FP64 (the FP32 entries are exact in FP64), so the decision Psi < mu is
// taken in FP64.  One wave scores one node: the subset is drawn by lane 0
// into LDS, then 64 lanes span the embedding dimension.
//
// The next active set keeps the scored nodes with Psi < mu, in their order
// (a sorted list stays sorted), by an order-preserving compaction.
#include <cmath>

#include "common.h"
#include "scan.h"

namespace felog {

constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ double wave_sum_d(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

template <int VPL>
__global__ __launch_bounds__(256) void psi_kernel(
    const float* __restrict__ tin, const int64_t* __restrict__ indptr,
    const int32_t* __restrict__ indices, const int32_t* __restrict__ nodes, int64_t count,
    int32_t k_s, uint64_t seed, uint32_t round, double mu, double* __restrict__ psi,
    uint8_t* __restrict__ keep)
{
    constexpr int D = 64 * VPL;
    __shared__ int32_t picks[kWavesPerBlock][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    // block-uniform trip count, so the block barrier below is reached by all waves
    for (int64_t base = (int64_t)blockIdx.x * kWavesPerBlock; base < count;
         base += (int64_t)gridDim.x * kWavesPerBlock) {
        const int64_t i = base + wv;
        const bool live = i < count;
        const int32_t v = live ? (nodes ? nodes[i] : (int32_t)i) : 0;
        const int64_t lo = indptr[v];
        const int64_t deg = live ? indptr[v + 1] - lo : 0;
        int m = 0;
        if (deg > 0) {
            if (deg <= k_s) {
                m = (int)deg;
                if (lane < m) picks[wv][lane] = lane;
            } else {
                m = k_s;
                if (lane == 0) {
                    Rand4 r{};
                    for (int s = 0; s < k_s; ++s) {
                        const int64_t j = deg - k_s + s;   // Floyd: j runs over deg-k .. deg-1
                        if ((s & 3) == 0)
                            r = philox4x32((uint32_t)v, round, (uint32_t)(s >> 2), kTagPsi, seed);
                        const uint32_t x = (s & 3) == 0 ? r.v[0] : (s & 3) == 1 ? r.v[1]
                                           : (s & 3) == 2 ? r.v[2] : r.v[3];
                        int32_t t = (int32_t)scale32(x, (uint32_t)(j + 1));   // uniform in [0, j]
                        bool seen = false;
                        for (int q = 0; q < s; ++q) seen |= picks[wv][q] == t;
                        picks[wv][s] = seen ? (int32_t)j : t;
                    }
                }
            }
        }
        __syncthreads();
        if (live) {
            if (deg == 0) {
                if (lane == 0) {
                    psi[i] = __longlong_as_double(0x7FF8000000000000ll);   // NaN
                    keep[i] = 0;
                }
            } else {
                double a[VPL];
                double na = 0.0;
#pragma unroll
                for (int e = 0; e < VPL; ++e) {
                    a[e] = (double)tin[(int64_t)v * D + e * 64 + lane];
                    na += a[e] * a[e];
                }
                na = wave_sum_d(na);
                double acc = 0.0;
                for (int s = 0; s < m; ++s) {
                    const int32_t u = indices[lo + picks[wv][s]];
                    double dot = 0.0, nb = 0.0;
#pragma unroll
                    for (int e = 0; e < VPL; ++e) {
                        double b = (double)tin[(int64_t)u * D + e * 64 + lane];
                        dot += a[e] * b;
                        nb += b * b;
                    }
                    dot = wave_sum_d(dot);
                    nb = wave_sum_d(nb);
                    acc += (na == 0.0 || nb == 0.0) ? 0.0 : dot / (sqrt(na) * sqrt(nb));
                }
                const double p = acc / (double)m;
                if (lane == 0) {
                    psi[i] = p;
                    keep[i] = p < mu ? 1 : 0;
                }
            }
        }
        __syncthreads();
    }
}

struct Kept {
    const uint8_t* keep;
    __device__ bool operator()(int64_t i) const { return keep[i] != 0; }
};
struct NodeAt {
    const int32_t* nodes;   // NULL: identity
    __device__ int32_t operator()(int64_t i) const { return nodes ? nodes[i] : (int32_t)i; }
};

void feedback(Model& m, const felog_feedback_params& p, const Active* in, Active& out,
              double* psi_host, int64_t psi_cap)
{
    Ctx& c = *m.ctx;
    c.make_current();
    const Graph& g = *m.g;
    const int64_t count = in ? in->count : g.n;
    const int32_t* nodes = in ? in->nodes.as<int32_t>() : nullptr;
    out.g = const_cast<Graph*>(&g);
    if (count == 0) {
        out.count = 0;
        out.nodes.alloc(&c, sizeof(int32_t));
        return;
    }
    DevBuf psi, keep;
    psi.alloc(&c, sizeof(double) * count);
    keep.alloc(&c, sizeof(uint8_t) * count);
    int64_t blocks = std::min<int64_t>((count + kWavesPerBlock - 1) / kWavesPerBlock,
                                       (int64_t)c.num_cus * 16);
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3((uint32_t)blocks), dim3(64 * kWavesPerBlock), 0,
                           c.stream, m.tin.as<float>(), g.indptr.as<int64_t>(),
                           g.indices.as<int32_t>(), nodes, count, p.k_s, p.seed, p.round, p.mu,
                           psi.as<double>(), keep.as<uint8_t>());
    };
    if (m.dim == 64) launch(psi_kernel<1>);
    else if (m.dim == 128) launch(psi_kernel<2>);
    else launch(psi_kernel<4>);
    FELOG_HIP(hipGetLastError());
    out.count = compact(c, Kept{keep.as<uint8_t>()}, NodeAt{nodes}, count, out.nodes);
    if (psi_host) {
        FELOG_REQUIRE(psi_cap >= count, "psi buffer holds %lld values, need %lld",
                      (long long)psi_cap, (long long)count);
        FELOG_HIP(hipMemcpyAsync(psi_host, psi.ptr, sizeof(double) * count,
                                 hipMemcpyDeviceToHost, c.stream));
    }
    c.sync();
}

int64_t compact_nodes(Ctx& ctx, const int32_t* d_nodes, const uint8_t* d_flags, int64_t count,
                      DevBuf& out)
{
    return compact(ctx, Kept{d_flags}, NodeAt{d_nodes}, count, out);
}

}  // namespace felog
