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
#include <mutex>

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
    uint8_t* keep /* nullable */)
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
                    if (keep) keep[i] = 0;
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
                    if (keep) keep[i] = p < mu ? 1 : 0;
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

static void launch_psi(Model& m, const felog_feedback_params& p, const int32_t* nodes,
                       int64_t count, double* psi, uint8_t* keep)
{
    Ctx& c = *m.ctx;
    const Graph& g = *m.g;
    int64_t blocks = std::min<int64_t>((count + kWavesPerBlock - 1) / kWavesPerBlock,
                                       (int64_t)c.num_cus * 16);
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3((uint32_t)blocks), dim3(64 * kWavesPerBlock), 0,
                           c.stream, m.tin.as<float>(), g.indptr.as<int64_t>(),
                           g.indices.as<int32_t>(), nodes, count, p.k_s, p.seed, p.round, p.mu,
                           psi, keep);
    };
    if (m.dim == 64) launch(psi_kernel<1>);
    else if (m.dim == 128) launch(psi_kernel<2>);
    else launch(psi_kernel<4>);
    FELOG_HIP(hipGetLastError());
}

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
    launch_psi(m, p, nodes, count, psi.as<double>(), keep.as<uint8_t>());
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

// ---------------------------------------------------------------------------
// The same feedback step without any device allocation, for callers that
// cannot allocate (code under graph capture, tight serving loops).  Psi goes
// to the caller's buffer and decides the next set (Psi < mu, NaN never kept),
// so the only scratch is the compaction's per-block counts and an input
// check flag, in a fixed array each device holds for the life of the process.
// ---------------------------------------------------------------------------
constexpr int64_t kNoallocMaxNodes = (int64_t)1 << 24;
constexpr int64_t kNoallocBlocksMax = (kNoallocMaxNodes + kScanSpan - 1) / kScanSpan;
// word 0: the input-check flag; words 64 ..: the compaction's block counts and total
constexpr int64_t kNoallocCountsAt = 64;
constexpr int64_t kNoallocWords = kNoallocCountsAt + kNoallocBlocksMax + 1;

static __device__ __align__(256) uint32_t scratch[kNoallocWords];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};   // per device: scratch's device address
}  // namespace

void noalloc_scratch_init(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    FELOG_REQUIRE(device >= 0 && device < 64, "device %d out of range", device);
    if (g_scratch_ptr[device]) return;
    void* ptr = nullptr;
    FELOG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    FELOG_REQUIRE(ptr != nullptr, "no device address for the feedback scratch array");
    g_scratch_ptr[device] = ptr;
}

static uint32_t* noalloc_scratch(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    FELOG_REQUIRE(device >= 0 && device < 64 && g_scratch_ptr[device],
                  "feedback scratch not set up on device %d", device);
    return static_cast<uint32_t*>(g_scratch_ptr[device]);
}

// flag = 1 if nodes[0, count) is not strictly increasing within [0, n)
__global__ __launch_bounds__(256) void check_nodes_kernel(const int32_t* nodes, int64_t count,
                                                           int32_t n, uint32_t* flag)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * 256) {
        const int32_t v = nodes[i];
        if (v < 0 || v >= n || (i > 0 && nodes[i - 1] >= v)) *flag = 1u;
    }
}

__global__ void clear_word_kernel(uint32_t* w) { *w = 0u; }

struct PsiBelow {
    const double* psi;
    double mu;
    __device__ bool operator()(int64_t i) const { return psi[i] < mu; }
};

void feedback_noalloc(Model& m, const felog_feedback_params& p, const int32_t* in_nodes,
                      int64_t count, int32_t* out_nodes, int64_t out_cap, double* psi,
                      int64_t psi_cap, int64_t* out_count)
{
    Ctx& c = *m.ctx;
    c.make_current();
    const Graph& g = *m.g;
    const bool all = p.mode == FELOG_FEEDBACK_RECOMPUTE_ALL || in_nodes == nullptr;
    const int32_t* nodes = all ? nullptr : in_nodes;
    const int64_t scored = all ? g.n : count;
    FELOG_REQUIRE(scored <= kNoallocMaxNodes, "the allocation-free feedback scores at most %lld "
                  "nodes (%lld asked)", (long long)kNoallocMaxNodes, (long long)scored);
    FELOG_REQUIRE(psi && psi_cap >= scored, "psi buffer holds %lld values, need %lld",
                  (long long)psi_cap, (long long)scored);
    FELOG_REQUIRE(out_nodes || scored == 0, "out_nodes is NULL");
    FELOG_REQUIRE(out_cap >= scored, "out_nodes holds %lld ids, need up to %lld",
                  (long long)out_cap, (long long)scored);
    uint32_t* sc = noalloc_scratch(c.device);
    *out_count = 0;
    if (scored == 0) return;
    if (nodes) {
        // the scored list must be valid before any kernel reads rows through it
        uint32_t bad = 0;
        hipLaunchKernelGGL(clear_word_kernel, dim3(1), dim3(1), 0, c.stream, sc);
        const int64_t blocks = std::min<int64_t>((scored + 255) / 256, (int64_t)c.num_cus * 4);
        hipLaunchKernelGGL(check_nodes_kernel, dim3((uint32_t)blocks), dim3(256), 0, c.stream,
                           nodes, scored, g.n, sc);
        FELOG_HIP(hipGetLastError());
        FELOG_HIP(hipMemcpyAsync(&bad, sc, sizeof bad, hipMemcpyDeviceToHost, c.stream));
        c.sync();
        FELOG_REQUIRE(bad == 0, "in_nodes must be strictly increasing node ids in [0, n)");
    }
    launch_psi(m, p, nodes, scored, psi, nullptr);
    // order-preserving compaction with the counts in scratch (every word the
    // passes read is written first: no clearing needed)
    const int64_t nb = (scored + kScanSpan - 1) / kScanSpan;
    uint32_t* counts = sc + kNoallocCountsAt;
    const PsiBelow pred{psi, p.mu};
    const NodeAt val{nodes};
    hipLaunchKernelGGL(compact_count_kernel<PsiBelow>, dim3((uint32_t)nb), dim3(kScanThreads), 0,
                       c.stream, pred, scored, counts);
    hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(kScanThreads), 0, c.stream, counts, nb);
    hipLaunchKernelGGL((compact_scatter_kernel<PsiBelow, NodeAt>), dim3((uint32_t)nb),
                       dim3(kScanThreads), 0, c.stream, pred, val, scored, counts, out_nodes);
    FELOG_HIP(hipGetLastError());
    uint32_t total = 0;
    FELOG_HIP(hipMemcpyAsync(&total, counts + nb, sizeof total, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    *out_count = total;
}

}  // namespace felog
