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
// Per minibatch two kernels run:
//   forward: per pair, gather in[ctx], out[ctr] and K noise rows, K+1 dot
//            products, sigma, coefficients g, and scatter-add the row deltas
//            into zeroed delta tables with FP32 atomics; first touches of a
//            row in this minibatch append it to a touched list (stamps).
//   apply:   for each touched row, table += delta, delta = 0.
// The tables are only read during forward, so every pair sees the state at
// the start of the minibatch, and the sum of a row's deltas is added once.
//
// A wave owns up to 64/(K+2) pairs: pair metadata, noise draws and stamps are
// computed for all of them at once in parallel lanes, then rows are processed
// pair by pair with 64 lanes spanning d (lane owns elements lane + 64 v).
#include <algorithm>

#include "common.h"
#include "noise.h"

namespace felog {

struct SgnsArgs {
    const float* __restrict__ tin;
    const float* __restrict__ tout;
    float* din;
    float* dout;
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
    uint32_t serial;
    uint32_t* stamp_in;
    uint32_t* stamp_out;
    int32_t* list_in;
    int32_t* list_out;
    uint32_t* cnt;                        // [0] in-list length, [1] out-list length
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

template <int VPL, int K>
__global__ __launch_bounds__(256) void sgns_forward_kernel(SgnsArgs a)
{
    constexpr int D = 64 * VPL;
    const int lane = threadIdx.x & 63;
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

    // ---- first-touch stamps and touched lists: lane l < np*(K+2) handles
    //      row r = l % (K+2) of pair l / (K+2): r = 0 centre, 1..K negatives
    //      (out table), K+1 context (in table).
    {
        const int p = lane / (K + 2);
        const int r = lane - p * (K + 2);
        const int ps = p < np ? p : 0;
        int32_t ctr = __shfl(m_ctr, ps);
        int32_t ctx = __shfl(m_ctx, ps);
        int32_t neg = __shfl(m_neg, ps * K + (r >= 1 && r <= K ? r - 1 : 0));
        int which = -1;   // 1 = out table, 0 = in table
        int32_t row = 0;
        if (lane < np * (K + 2)) {
            if (r == 0) { which = 1; row = ctr; }
            else if (r <= K) { which = neg != ctr ? 1 : -1; row = neg; }
            else { which = 0; row = ctx; }
        }
        uint32_t old = a.serial;
        if (which == 1) old = atomicExch(&a.stamp_out[row], a.serial);
        else if (which == 0) old = atomicExch(&a.stamp_in[row], a.serial);
        const bool fresh = which >= 0 && old != a.serial;
        const uint64_t bout = __ballot(fresh && which == 1);
        const uint64_t bin = __ballot(fresh && which == 0);
        uint32_t base_out = 0, base_in = 0;
        if (lane == 0) {
            if (bout) base_out = atomicAdd(&a.cnt[1], (uint32_t)__popcll(bout));
            if (bin) base_in = atomicAdd(&a.cnt[0], (uint32_t)__popcll(bin));
        }
        base_out = __shfl(base_out, 0);
        base_in = __shfl(base_in, 0);
        const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
        if (fresh && which == 1) a.list_out[base_out + __popcll(bout & below)] = row;
        if (fresh && which == 0) a.list_in[base_in + __popcll(bin & below)] = row;
    }

    // ---- rows, dots, coefficients and scatter-add, one pair at a time
    float s_term = 0.0f;
    bool s_valid = false;
    for (int p = 0; p < np; ++p) {
        const int32_t ctx = __builtin_amdgcn_readlane(m_ctx, p);
        int32_t t[K + 1];
        t[0] = __builtin_amdgcn_readlane(m_ctr, p);
#pragma unroll
        for (int k = 0; k < K; ++k) t[k + 1] = __builtin_amdgcn_readlane(m_neg, p * K + k);

        float vin[VPL];
        float vo[K + 1][VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) vin[v] = a.tin[(int64_t)ctx * D + v * 64 + lane];
#pragma unroll
        for (int k = 0; k <= K; ++k)
#pragma unroll
            for (int v = 0; v < VPL; ++v) vo[k][v] = a.tout[(int64_t)t[k] * D + v * 64 + lane];

        float dot[K + 1];
#pragma unroll
        for (int k0 = 0; k0 <= K; k0 += 8) {
            float part[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                part[i] = 0.0f;
                if (k0 + i <= K) {
#pragma unroll
                    for (int v = 0; v < VPL; ++v) part[i] = fmaf(vin[v], vo[k0 + i][v], part[i]);
                }
            }
            float red = reduce8(part, lane);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (k0 + i <= K) dot[k0 + i] = __shfl(red, 8 * i);
        }

        float g[K + 1];
        g[0] = a.lr * (1.0f - sigmoidf_(dot[0]));
#pragma unroll
        for (int k = 1; k <= K; ++k) g[k] = t[k] != t[0] ? -a.lr * sigmoidf_(dot[k]) : 0.0f;

        // loss terms for this pair go to lanes p*(K+1) .. p*(K+1)+K
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            if (lane == p * (K + 1) + k) {
                s_term = k == 0 ? -dot[0] : dot[k];
                s_valid = k == 0 || t[k] != t[0];
            }
        }

        float dctx[VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k <= K; ++k) acc = fmaf(g[k], vo[k][v], acc);
            dctx[v] = acc;
        }
#pragma unroll
        for (int v = 0; v < VPL; ++v)
            unsafeAtomicAdd(&a.din[(int64_t)ctx * D + v * 64 + lane], dctx[v]);
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            if (k > 0 && t[k] == t[0]) continue;
#pragma unroll
            for (int v = 0; v < VPL; ++v)
                unsafeAtomicAdd(&a.dout[(int64_t)t[k] * D + v * 64 + lane], g[k] * vin[v]);
        }
    }

    // ---- loss: -log sigma(s0) - sum_k log sigma(-s_k) = softplus(-s0) + sum_k softplus(s_k)
    double term = s_valid ? neg_log_sigmoid(-(double)s_term) : 0.0;
    term = wave_sum_f64(term);
    if (lane == 0) a.loss_part[gwave] += term;
}

template <int VPL>
__global__ __launch_bounds__(256) void sgns_apply_kernel(float* __restrict__ tin,
                                                         float* __restrict__ tout,
                                                         float* __restrict__ din,
                                                         float* __restrict__ dout,
                                                         const int32_t* __restrict__ list_in,
                                                         const int32_t* __restrict__ list_out,
                                                         const uint32_t* cnt, uint32_t* cnt_next,
                                                         unsigned long long* row_totals)
{
    constexpr int D = 64 * VPL;
    const int lane = threadIdx.x & 63;
    const uint32_t n_in = cnt[0], n_out = cnt[1];
    const uint32_t total = n_in + n_out;
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    for (uint32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < total; i += nw) {
        const bool is_in = i < n_in;
        const int32_t row = is_in ? list_in[i] : list_out[i - n_in];
        float* T = is_in ? tin : tout;
        float* Dl = is_in ? din : dout;
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            int64_t idx = (int64_t)row * D + v * 64 + lane;
            T[idx] += Dl[idx];
            Dl[idx] = 0.0f;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cnt_next[0] = 0;
        cnt_next[1] = 0;
        row_totals[0] += n_in;
        row_totals[1] += n_out;
    }
}

// Copy the deltas of the touched rows out (row-major [count][D]) and clear them.
template <int VPL>
__global__ void sgns_capture_kernel(float* __restrict__ delta, const int32_t* __restrict__ list,
                                    uint32_t count, float* __restrict__ out,
                                    int32_t* __restrict__ rows)
{
    constexpr int D = 64 * VPL;
    const int lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    for (uint32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < count; i += nw) {
        int32_t row = list[i];
        if (lane == 0) rows[i] = row;
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            int64_t idx = (int64_t)row * D + v * 64 + lane;
            out[(int64_t)i * D + v * 64 + lane] = delta[idx];
            delta[idx] = 0.0f;
        }
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
template <int VPL, int K>
static void launch_forward_t(dim3 grid, hipStream_t s, const SgnsArgs& a)
{
    hipLaunchKernelGGL((sgns_forward_kernel<VPL, K>), grid, dim3(256), 0, s, a);
}

template <int VPL>
static void launch_forward_k(int K, dim3 grid, hipStream_t s, const SgnsArgs& a)
{
    switch (K) {
#define FELOG_K(k) case k: launch_forward_t<VPL, k>(grid, s, a); break;
        FELOG_K(1) FELOG_K(2) FELOG_K(3) FELOG_K(4) FELOG_K(5) FELOG_K(6) FELOG_K(7)
        FELOG_K(8) FELOG_K(9) FELOG_K(10) FELOG_K(11) FELOG_K(12) FELOG_K(13) FELOG_K(14)
        FELOG_K(15) FELOG_K(16) FELOG_K(17) FELOG_K(18) FELOG_K(19) FELOG_K(20)
#undef FELOG_K
        default: fail(FELOG_EUNSUPPORTED, "negatives = %d not supported", K);
    }
}

static void launch_forward(int dim, int K, dim3 grid, hipStream_t s, const SgnsArgs& a)
{
    if (dim == 64) launch_forward_k<1>(K, grid, s, a);
    else if (dim == 128) launch_forward_k<2>(K, grid, s, a);
    else launch_forward_k<4>(K, grid, s, a);
    FELOG_HIP(hipGetLastError());
}

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

struct Schedule {
    std::vector<int64_t> chunk_first_mb;   // first global minibatch of each chunk
    std::vector<int64_t> chunk_pairs;
    std::vector<int64_t> chunk_valid_base; // offset of the chunk in valid_cols
    int64_t B = 0;
    int64_t total_pairs = 0;
    int64_t nslices = 0;
};

static Schedule make_schedule(Walks& w, const felog_train_params& p)
{
    int64_t chunk = p.chunk_walks ? p.chunk_walks : (int64_t)1 << 20;
    launch_valid_columns(w, chunk);
    Schedule s;
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
    Schedule s = make_schedule(w, p);
    if (total_pairs) *total_pairs = s.total_pairs;
    return s.B;
}

void train_minibatches(Model& m, const Walks& wc, const felog_train_params& p, int64_t first_mb,
                       int64_t n_mb, bool apply, felog_train_stats* stats, int32_t* rows_in,
                       float* d_in_host, int64_t cap_in, int64_t* n_in, int32_t* rows_out,
                       float* d_out_host, int64_t cap_out, int64_t* n_out)
{
    Walks& w = const_cast<Walks&>(wc);
    Ctx& c = *m.ctx;
    c.make_current();
    Schedule sch = make_schedule(w, p);
    const int K = p.negatives;
    const int64_t P = p.minibatch_pairs;
    int64_t end = n_mb < 0 ? sch.B : std::min<int64_t>(sch.B, first_mb + n_mb);
    if (first_mb > sch.B) first_mb = sch.B;
    if (!apply) FELOG_REQUIRE(first_mb < sch.B, "minibatch %lld out of range (%lld minibatches)",
                              (long long)first_mb, (long long)sch.B);

    // scratch sized for this minibatch size
    if (m.cap_pairs < P || m.cap_K < K) {
        m.cap_pairs = std::max<int64_t>(m.cap_pairs, P);
        m.cap_K = std::max(m.cap_K, K);
        m.touched_in.alloc(&c, sizeof(int32_t) * m.cap_pairs);
        m.touched_out.alloc(&c, sizeof(int32_t) * m.cap_pairs * (m.cap_K + 1));
    }
    const int ppw_max = 64 / (K + 2);
    int ppw = (int)std::min<int64_t>(ppw_max, std::max<int64_t>(1, P / ((int64_t)c.num_cus * 32)));
    const int64_t waves = (P + ppw - 1) / ppw;
    const int64_t blocks = (waves + 3) / 4;
    DevBuf loss_part;
    loss_part.alloc(&c, sizeof(double) * blocks * 4);
    FELOG_HIP(hipMemsetAsync(loss_part.ptr, 0, sizeof(double) * blocks * 4, c.stream));
    FELOG_HIP(hipMemsetAsync(m.counters.ptr, 0, sizeof(uint32_t) * 4, c.stream));
    FELOG_HIP(hipMemsetAsync(m.row_totals.ptr, 0, sizeof(uint64_t) * 2, c.stream));

    // sampled kernel timing: events before forward, between forward and apply, after apply
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
    a.din = m.din.as<float>();
    a.dout = m.dout.as<float>();
    a.walks = w.data.as<int32_t>();
    a.W = w.W;
    a.slices = slices.as<int32_t>();
    a.id_base = w.id_base;
    a.window = p.window;
    a.ppw = ppw;
    a.seed = p.seed;
    a.noise = NoiseTable{m.cdf.as<uint64_t>(), m.guide.as<int32_t>(), m.total_weight, m.guide_bits};
    a.stamp_in = m.stamp_in.as<uint32_t>();
    a.stamp_out = m.stamp_out.as<uint32_t>();
    a.list_in = m.touched_in.as<int32_t>();
    a.list_out = m.touched_out.as<int32_t>();
    a.loss_part = loss_part.as<double>();

    const double lr0 = (double)p.lr_start, lr1 = (double)p.lr_end;
    const int apply_blocks = std::max(1, c.num_cus * 8);
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
        const int parity = (int)(m.serial & 1u);
        a.serial = m.serial;
        a.cnt = m.counters.as<uint32_t>() + 2 * parity;
        int64_t nwaves = (np + ppw - 1) / ppw;
        const bool timed_mb = every > 0 && pool > 0 && (b - first_mb) % every == 0;
        hipEvent_t* ev = nullptr;
        if (timed_mb) {
            if (used_slots == pool) harvest(next_slot);   // reuse the oldest slot
            else ++used_slots;
            ev = &c.timing_pool[3 * next_slot];
            next_slot = (next_slot + 1) % pool;
            FELOG_HIP(hipEventRecord(ev[0], c.stream));
        }
        launch_forward(m.dim, K, dim3((uint32_t)((nwaves + 3) / 4)), c.stream, a);
        if (timed_mb) FELOG_HIP(hipEventRecord(ev[1], c.stream));
        if (apply) {
            uint32_t* next = m.counters.as<uint32_t>() + 2 * (1 - parity);
            if (m.dim == 64)
                hipLaunchKernelGGL(sgns_apply_kernel<1>, dim3(apply_blocks), dim3(256), 0,
                                   c.stream, m.tin.as<float>(), m.tout.as<float>(), a.din,
                                   a.dout, a.list_in, a.list_out, a.cnt, next,
                                   m.row_totals.as<unsigned long long>());
            else if (m.dim == 128)
                hipLaunchKernelGGL(sgns_apply_kernel<2>, dim3(apply_blocks), dim3(256), 0,
                                   c.stream, m.tin.as<float>(), m.tout.as<float>(), a.din,
                                   a.dout, a.list_in, a.list_out, a.cnt, next,
                                   m.row_totals.as<unsigned long long>());
            else
                hipLaunchKernelGGL(sgns_apply_kernel<4>, dim3(apply_blocks), dim3(256), 0,
                                   c.stream, m.tin.as<float>(), m.tout.as<float>(), a.din,
                                   a.dout, a.list_in, a.list_out, a.cnt, next,
                                   m.row_totals.as<unsigned long long>());
            FELOG_HIP(hipGetLastError());
            if (timed_mb) FELOG_HIP(hipEventRecord(ev[2], c.stream));
        } else {
            uint32_t h_cnt[2];
            FELOG_HIP(hipMemcpyAsync(h_cnt, a.cnt, sizeof h_cnt, hipMemcpyDeviceToHost,
                                     c.stream));
            c.sync();
            FELOG_REQUIRE(rows_in && d_in_host && rows_out && d_out_host,
                          "capture buffers must not be NULL");
            FELOG_REQUIRE((int64_t)h_cnt[0] <= cap_in && (int64_t)h_cnt[1] <= cap_out,
                          "capture buffers hold %lld / %lld rows, need %u / %u",
                          (long long)cap_in, (long long)cap_out, h_cnt[0], h_cnt[1]);
            DevBuf vin, vout, rin, rout;
            vin.alloc(&c, sizeof(float) * (size_t)std::max(1u, h_cnt[0]) * m.dim);
            vout.alloc(&c, sizeof(float) * (size_t)std::max(1u, h_cnt[1]) * m.dim);
            rin.alloc(&c, sizeof(int32_t) * std::max(1u, h_cnt[0]));
            rout.alloc(&c, sizeof(int32_t) * std::max(1u, h_cnt[1]));
            auto cap = [&](float* delta, const int32_t* list, uint32_t count, DevBuf& vals,
                           DevBuf& rows) {
                if (!count) return;
                dim3 grid(std::min<uint32_t>((count + 3) / 4, 4096));
                if (m.dim == 64)
                    hipLaunchKernelGGL(sgns_capture_kernel<1>, grid, dim3(256), 0, c.stream, delta,
                                       list, count, vals.as<float>(), rows.as<int32_t>());
                else if (m.dim == 128)
                    hipLaunchKernelGGL(sgns_capture_kernel<2>, grid, dim3(256), 0, c.stream, delta,
                                       list, count, vals.as<float>(), rows.as<int32_t>());
                else
                    hipLaunchKernelGGL(sgns_capture_kernel<4>, grid, dim3(256), 0, c.stream, delta,
                                       list, count, vals.as<float>(), rows.as<int32_t>());
                FELOG_HIP(hipGetLastError());
            };
            cap(a.din, a.list_in, h_cnt[0], vin, rin);
            cap(a.dout, a.list_out, h_cnt[1], vout, rout);
            FELOG_HIP(hipMemcpyAsync(rows_in, rin.ptr, sizeof(int32_t) * h_cnt[0],
                                     hipMemcpyDeviceToHost, c.stream));
            FELOG_HIP(hipMemcpyAsync(rows_out, rout.ptr, sizeof(int32_t) * h_cnt[1],
                                     hipMemcpyDeviceToHost, c.stream));
            FELOG_HIP(hipMemcpyAsync(d_in_host, vin.ptr, sizeof(float) * h_cnt[0] * m.dim,
                                     hipMemcpyDeviceToHost, c.stream));
            FELOG_HIP(hipMemcpyAsync(d_out_host, vout.ptr, sizeof(float) * h_cnt[1] * m.dim,
                                     hipMemcpyDeviceToHost, c.stream));
            FELOG_HIP(hipMemsetAsync(m.counters.ptr, 0, sizeof(uint32_t) * 4, c.stream));
            c.sync();
            if (n_in) *n_in = h_cnt[0];
            if (n_out) *n_out = h_cnt[1];
        }
        ++m.serial;
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
