// Skip-gram with negative sampling for small minibatches (Train of
// Algorithm 1; Eq. (1)-(2)): P (K + 2) <= 8192 touches per minibatch, the
// shape of the 1,024-pair configurations.
//
// At that size a minibatch moves a few MB, so the per-minibatch launch chain
// of sgns.hip (ids, two scan passes, forward, two apply launches) is bound by
// launch and cache-flush latency, not by HBM.  Here the work splits in two:
//
//   plan    one workgroup per minibatch, many minibatches per launch.  It
//           draws the minibatch's node ids (walk reads, noise draws), sorts
//           its touches by (table, row, touch) with a bitonic network in LDS
//           and lists the rows' segments.  Sorting by touch index within a
//           row is pair order (pair, then slot), so no atomics and no
//           per-row counters are needed.  Plans depend only on the walks and
//           the noise table, never on the embeddings.
//   update  one persistent cooperative launch for those minibatches.  Per
//           minibatch: the forward (gathers, FP64 dots, sigma, coefficients;
//           each out-touch's coefficient at its sorted position; the context
//           row copied for pairs with an out row touched more than once; rows
//           touched once in either table updated in place), a grid barrier,
//           the apply (one 16-lane group per segment of two or more touches
//           sums the row's terms and adds them once), and a grid barrier.
//           The apply reads the context copies, not the in-table, so in and
//           out rows are applied together.
//
// The arithmetic is that of sgns.hip term for term: rows of at most kChunk
// touches sum their FP64 terms sequentially in pair order, longer rows sum
// terms rounded onto the exact-sum grid, every stored value is rounded once.
// The two paths therefore give bit-identical tables.
//
// The grid barrier is a flag per workgroup: each workgroup stores its barrier
// count to a flag on its own 128-byte line, and the first wave of every
// workgroup watches all the flags (one lane per flag).  On MI355X (512
// threads per workgroup) this measured 1.7 us at 32 workgroups, 2.2 at 64 and
// 3.4 at 128; workgroup 0 gathering the flags and raising a go flag that the
// others wait for took 2.0-3.1 / 2.5 / 3.5 us, and one shared atomic counter,
// whose same-address atomics serialise, 3.4 / 3.4 / 4.9 us.  Every wait is
// bounded: one that exceeds kSpinLimit polls raises an abort flag that every
// workgroup checks, so every wave leaves the kernel, and the host reports the
// failure.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "noise.h"
#include "sgns_device.h"

namespace felog {

// Values of one minibatch that the plan and update launches read.
struct MbDesc {
    int64_t vcol_base;     // offset of the minibatch's chunk in valid_cols
    uint32_t Wv;           // valid columns of the chunk
    uint32_t first_pair;   // first pair of the minibatch in its chunk
    uint32_t npairs;
    float lr;
    double grid_c;         // exact-sum grid constant of lr
};
static_assert(sizeof(MbDesc) == 32, "descriptor layout shared by host and device");

constexpr int kPlanThreads = 512;
constexpr int kPlanMaxTouches = kSmallMaxTouches;   // touches a plan sorts in LDS (64 KB of keys)
constexpr int32_t kPosMask = (1 << 30) - 1;
constexpr int32_t kSingleBit = 1 << 30;  // row touched once in the minibatch: the forward updates it
constexpr uint32_t kSpinLimit = 1u << 22;  // polls before a barrier wait gives up (seconds)
constexpr int kUpdThreads = 512;         // one workgroup per CU at two waves per SIMD
constexpr int kFlagStride = 32;          // 32-bit words between barrier flags (128 bytes)
constexpr int kDefaultUpdBlocks = 64;    // workgroups of the persistent launch by default

// ------------------------------------------------------------------- plan
struct PlanArgs {
    const int32_t* walks;          // step-major [L][W]
    int64_t W;
    const int32_t* vcols;
    const int32_t* slices;         // (j << 8) | slot
    int64_t id_base;
    int32_t window;
    uint64_t seed;
    NoiseTable noise;
    const MbDesc* desc;            // [minibatches of the launch]
    int32_t tmax;                  // touch slots per minibatch, P (K + 2)
    int2* tinfo;                   // [mb][tmax]: (row, sorted position | kSingleBit), -1 skipped
    int4* segs;                    // [mb][tmax]: (row, first position, touches, table)
    int32_t* spair;                // [mb][tmax]: pair of each sorted position
    uint32_t* meta;                // [mb][4]: applied segments, applied in segments,
                                   // out rows, out rows touched once
    unsigned long long* row_totals;// [3]: in rows, out rows, out rows touched once
};

// Plans of one launch: workgroups [start[j], start[j + 1]) plan the
// minibatches of job j (one model and corpus per job).
struct PlanBatch {
    PlanArgs job[kMaxBatchJobs];
    int32_t start[kMaxBatchJobs + 1];
    int32_t njobs;
};

// Exclusive scan of one value per thread over the workgroup; *total gets the sum.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* tmp, uint32_t* total)
{
    constexpr int NW = kPlanThreads / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) tmp[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < NW; ++i) {
            const uint32_t c = tmp[i];
            tmp[i] = run;
            run += c;
        }
        tmp[NW] = run;
    }
    __syncthreads();
    const uint32_t excl = tmp[w] + x - v;
    *total = tmp[NW];
    __syncthreads();
    return excl;
}

template <int K>
__global__ __launch_bounds__(kPlanThreads) void sgns_plan_kernel(PlanBatch pb)
{
    constexpr int T = K + 2;
    int jb = 0;
    while (jb + 1 < pb.njobs && (int32_t)blockIdx.x >= pb.start[jb + 1]) ++jb;
    const PlanArgs& a = pb.job[jb];
    const uint32_t lb = blockIdx.x - (uint32_t)pb.start[jb];   // minibatch within the job's group
    __shared__ unsigned long long keys[kPlanMaxTouches];
    // segment starts (step 3); before that, the pairs' centres (step 1)
    __shared__ __align__(16) uint16_t seg_first[kPlanMaxTouches + 1];
    __shared__ uint32_t tmp[kPlanThreads / 64 + 1];
    __shared__ uint32_t counts[3];     // in rows, out rows touched once, applied in segments
    const MbDesc d = a.desc[lb];
    const uint32_t nt = d.npairs * T;
    uint32_t N = 64;
    while (N < nt) N <<= 1;                 // nt <= kPlanMaxTouches (checked on the host)
    int2* tinfo = a.tinfo + (int64_t)lb * a.tmax;
    int4* segs = a.segs + (int64_t)lb * a.tmax;
    int32_t* spair = a.spair + (int64_t)lb * a.tmax;
    const int32_t* vcols = a.vcols + d.vcol_base;
    if (threadIdx.x < 3) counts[threadIdx.x] = 0;

    // 1. each touch's row and sort key (table << 62 | row << 16 | touch).  A
    //    pair's walk reads are made once: its context and centre first (one
    //    thread per pair), then the negatives (one thread per negative),
    //    which read the centre from LDS; every thread's loads are independent
    //    of its earlier items', so they overlap.
    for (uint32_t t = threadIdx.x; t < N; t += kPlanThreads) keys[t] = ~0ull;
    __syncthreads();
    int32_t* ctr_of = reinterpret_cast<int32_t*>(seg_first);   // [P] centres, until step 3
    for (uint32_t p = threadIdx.x; p < d.npairs; p += kPlanThreads) {
        const uint32_t gq = d.first_pair + p;
        const uint32_t sidx = gq / d.Wv;
        const uint32_t rank = gq - sidx * d.Wv;
        const int32_t js = a.slices[sidx];
        const int32_t col = vcols[rank];
        const int32_t j = js >> 8, s = js & 255;
        const int32_t off = s < a.window ? s - a.window : s - a.window + 1;
        const int32_t ctr = a.walks[(int64_t)j * a.W + col];
        const int32_t ctx = a.walks[(int64_t)(j + off) * a.W + col];
        ctr_of[p] = ctr;
        keys[p * T] = ((unsigned long long)ctx << 16) | (p * T);
        keys[p * T + 1] = (1ull << 62) | ((unsigned long long)ctr << 16) | (p * T + 1);
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < d.npairs * K; e += kPlanThreads) {
        // negative k of pair p: Philox(walk id, (j << 8) | slot, NEG | k / 2), words
        // 2 (k mod 2) and 2 (k mod 2) + 1
        const uint32_t p = e / K, k = e - p * K;
        const uint32_t gq = d.first_pair + p;
        const uint32_t sidx = gq / d.Wv;
        const uint32_t rank = gq - sidx * d.Wv;
        const int32_t js = a.slices[sidx];
        const int64_t wid = a.id_base + vcols[rank];
        const Rand4 x = philox4x32((uint32_t)wid, (uint32_t)(wid >> 32), (uint32_t)js,
                                   kTagNeg | (k >> 1), a.seed);
        const uint32_t lo = (k & 1) ? x.v[2] : x.v[0];
        const uint32_t hi = (k & 1) ? x.v[3] : x.v[1];
        const int32_t neg = noise_draw(a.noise, ((uint64_t)hi << 32) | lo);
        const uint32_t t = p * T + 2 + k;
        if (neg != ctr_of[p])
            keys[t] = (1ull << 62) | ((unsigned long long)neg << 16) | t;
        else
            tinfo[t] = make_int2(-1, -1);   // a negative equal to the centre is skipped
    }
    __syncthreads();

    // 2. bitonic sort, ascending
    for (uint32_t k = 2; k <= N; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < N; i += kPlanThreads) {
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

    // 3. segments: a position starts one where (table, row) changes; each
    //    thread takes a contiguous run of positions
    const uint32_t per = (N + kPlanThreads - 1) / kPlanThreads;
    const uint32_t lo = min(N, threadIdx.x * per), hi = min(N, lo + per);
    uint32_t nstart = 0, nvalid = 0;
    for (uint32_t i = lo; i < hi; ++i) {
        const unsigned long long x = keys[i];
        if (x == ~0ull) continue;
        ++nvalid;
        if (i == 0 || (keys[i - 1] >> 16) != (x >> 16)) ++nstart;
    }
    uint32_t nseg, nv;
    uint32_t s = block_scan(nstart, tmp, &nseg);
    block_scan(nvalid, tmp, &nv);
    for (uint32_t i = lo; i < hi; ++i) {
        const unsigned long long x = keys[i];
        if (x != ~0ull && (i == 0 || (keys[i - 1] >> 16) != (x >> 16))) seg_first[s++] = (uint16_t)i;
    }
    if (threadIdx.x == 0) seg_first[nseg] = (uint16_t)nv;
    __syncthreads();

    // 4. per segment: length; segments of two or more touches go to the
    //    apply list (in segments first: they sort first), rows touched once
    //    are updated by the forward; every touch's sorted position
    const uint32_t sper = (nseg + kPlanThreads - 1) / kPlanThreads;
    const uint32_t s_lo = min(nseg, threadIdx.x * sper), s_hi = min(nseg, s_lo + sper);
    uint32_t napply = 0, nin = 0, nin_apply = 0, nsingle = 0;
    for (uint32_t q = s_lo; q < s_hi; ++q) {
        const uint32_t f = seg_first[q], len = seg_first[q + 1] - f;
        const bool out = (keys[f] >> 62) != 0;
        napply += len > 1 ? 1u : 0u;
        nin += out ? 0u : 1u;
        nin_apply += (!out && len > 1) ? 1u : 0u;
        nsingle += (out && len == 1) ? 1u : 0u;
    }
    uint32_t n_apply;
    uint32_t slot = block_scan(napply, tmp, &n_apply);
    atomicAdd(&counts[0], nin);
    atomicAdd(&counts[1], nsingle);
    atomicAdd(&counts[2], nin_apply);
    for (uint32_t q = s_lo; q < s_hi; ++q) {
        const uint32_t f = seg_first[q], len = seg_first[q + 1] - f;
        const unsigned long long x = keys[f];
        const int32_t out = (int32_t)(x >> 62);
        const int32_t row = (int32_t)((x >> 16) & 0x7FFFFFFFull);
        const bool single = len == 1;
        if (!single) segs[slot++] = make_int4(row, (int32_t)f, (int32_t)len, out);
        for (uint32_t i = f; i < f + len; ++i) {
            const uint32_t t = (uint32_t)(keys[i] & 0xFFFF);
            tinfo[t] = make_int2(row, (int32_t)i | (single ? kSingleBit : 0));
            spair[i] = (int32_t)(t / T);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t* m = a.meta + (int64_t)lb * 4;
        m[0] = n_apply;
        m[1] = counts[2];
        m[2] = nseg - counts[0];
        m[3] = counts[1];
        atomicAdd(&a.row_totals[0], (unsigned long long)counts[0]);
        atomicAdd(&a.row_totals[1], (unsigned long long)(nseg - counts[0]));
        atomicAdd(&a.row_totals[2], (unsigned long long)counts[1]);
    }
}

// ----------------------------------------------------------------- update
// One job's part of an update launch.
struct UpdJob {
    float* tin;
    float* tout;
    const MbDesc* desc;            // [nmb]
    const int2* tinfo;             // [nmb][tmax]
    const int4* segs;              // [nmb][tmax]
    const uint32_t* meta;          // [nmb][4]
    const int32_t* spair;          // [nmb][tmax]: pair of each sorted position
    double* gpos;                  // [tmax]: FP64 coefficient of each out-touch, by position
    float* dinp;                   // [P][D]: each pair's in-row delta, by sorted position
    float* ctxc;                   // [P][D]: each pair's context row at the minibatch start
    double* loss_part;             // [waves]
    int32_t tmax;
    int32_t nmb;
};

// An update launch over the minibatches of up to kMaxBatchJobs jobs (equal d
// and K): phase by phase, minibatch m of every job that has one.  The jobs'
// tables are distinct, so their minibatches share each phase and its
// barriers.
struct UpdArgs {
    UpdJob job[kMaxBatchJobs];
    int32_t njobs;
    int32_t nmb_max;               // largest nmb of the jobs
    uint32_t* flags;               // workgroup b's at [kFlagStride (1 + b)] (the first line is
                                   // unused); zero at the call's start
    uint32_t epoch0;               // barriers passed by earlier launches of the call
    int32_t* abort;
    unsigned long long* clocks;    // null, or [4]: device wall-clock ticks of the forward,
                                   // the first barrier, the apply and the second barrier,
                                   // summed over workgroups and minibatches
};

// Bounded wait until *p >= target; false (and the abort flag raised) when
// the wait gives up or another workgroup has raised it.
__device__ __forceinline__ bool wait_at_least(const uint32_t* p, uint32_t target, int32_t* abort)
{
    uint32_t polls = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++polls > kSpinLimit) {
            __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((polls & 255) == 0 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Grid barrier with release/acquire at agent scope.  Returns false when the
// launch is aborting (a wait exceeded its bound somewhere).
__device__ __forceinline__ bool grid_sync(const UpdArgs& a, uint32_t& epoch,
                                          unsigned long long* arrive)
{
    __shared__ int s_ok;
    __syncthreads();
    if (arrive) *arrive = wall_clock64();   // every wave of the workgroup is here
    ++epoch;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&a.flags[kFlagStride * (1 + blockIdx.x)], epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    // every workgroup's first wave watches every flag (lane l the flags of
    // workgroups l, l + 64, ...), then acquires for the workgroup
    if (threadIdx.x < 64) {
        bool ok = true;
        for (uint32_t b = threadIdx.x; b < gridDim.x; b += 64)
            ok = ok && wait_at_least(&a.flags[kFlagStride * (1 + b)], epoch, a.abort);
        const bool all_ok = __all(ok);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (threadIdx.x == 0)
            s_ok = all_ok &&
                   !__hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return s_ok != 0;
}

template <int D, int K>
__global__ __launch_bounds__(kUpdThreads) void sgns_small_update_kernel(UpdArgs a)
{
    // lanes per pair in the forward: 32 at d >= 128, so that the 1,024 pairs of
    // a minibatch occupy every wave of the 64 workgroups (16 lanes left half
    // of them idle: 10.2 -> 6.8 us for the forward on R-MAT 2^20, K = 5)
    constexpr int LPP = D >= 128 ? 32 : 16;
    constexpr int G = 64 / LPP;                         // pairs in flight per wave
    constexpr int V4 = D / (4 * LPP);                   // float4s per lane and row
    constexpr int T = K + 2;
    constexpr int AV4 = D / 64;                         // float4s per lane and row (apply)
    constexpr int kRows = 4;                            // rows in flight per apply group
    const int lane = threadIdx.x & 63;
    const int grp = lane / LPP, gl = lane % LPP;
    const int g16 = lane >> 4, l16 = lane & 15;
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    const uint32_t gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    uint32_t epoch = a.epoch0;
    double lacc = 0.0;
    // plan data of job 0's next phase, loaded a phase ahead: this lane's touch
    // of the wave's first pair group (forward) and the group's first segment
    // with the pair of each of its first 16 positions (apply)
    const UpdJob& J0 = a.job[0];
    auto first_touch = [&](int mm) -> int2 {
        const uint32_t npm = J0.desc[mm].npairs, q0 = gw * G;
        if (q0 < npm && lane < (int)min((uint32_t)G, npm - q0) * T)
            return J0.tinfo[(int64_t)mm * J0.tmax + (int64_t)q0 * T + lane];
        return make_int2(-1, -1);
    };
    int2 pf_touch = J0.nmb > 0 ? first_touch(0) : make_int2(-1, -1);
    const uint32_t sidx0 = gw * 4 + (uint32_t)g16;

    // phase clocks (thread 0 of each workgroup, when asked for), kept in LDS:
    // [0..3] ticks of the phases summed over the launch's minibatches (added
    // to the totals once at the end), [4] phase start, [5] barrier arrival,
    // [6] first barrier's exit
    __shared__ unsigned long long s_clk[7];
    const bool clk = a.clocks != nullptr && threadIdx.x == 0;
    if (clk)
        for (int i = 0; i < 4; ++i) s_clk[i] = 0;
    for (int m = 0; m < a.nmb_max; ++m) {
        if (clk) s_clk[4] = wall_clock64();
        int4 pf_seg = make_int4(0, 0, 0, 0);
        int32_t pf_pair = 0;
        if (m < J0.nmb) {
            const uint32_t nseg0 = J0.meta[(int64_t)m * 4];
            if (sidx0 < nseg0) pf_seg = J0.segs[(int64_t)m * J0.tmax + sidx0];
        }

        // ---- forward of every job's minibatch m: G pairs per wave at a time
        for (int j = 0; j < a.njobs; ++j) {
            const UpdJob& J = a.job[j];
            if (m >= J.nmb) continue;
            const MbDesc dsc = J.desc[m];
            const int2* ti = J.tinfo + (int64_t)m * J.tmax;
            const uint32_t np = dsc.npairs;
            const double lr = (double)dsc.lr;
            for (uint32_t q0 = gw * G; q0 < np; q0 += nw * G) {
                const int npw = (int)min((uint32_t)G, np - q0);
                int32_t m_row = -1, m_code = -1;
                if (j == 0 && q0 == gw * G) {
                    m_row = pf_touch.x;
                    m_code = pf_touch.y;
                } else if (lane < npw * T) {
                    const int2 x = ti[(int64_t)q0 * T + lane];
                    m_row = x.x;
                    m_code = x.y;
                }
                const unsigned long long single = __ballot(m_code >= 0 && (m_code & kSingleBit));
                const int p = grp;
                const bool live = p < npw;
                const uint32_t q = q0 + (uint32_t)p;
                const int src = (live ? p : 0) * T;
                const int32_t ctx = __shfl(m_row, src);
                const int32_t pos_in = __shfl(m_code, src) & kPosMask;
                int32_t t[K + 1];
#pragma unroll
                for (int k = 0; k <= K; ++k) t[k] = __shfl(m_row, src + 1 + k);
                const int32_t my_code = __shfl(m_code, src + 1 + (gl <= K ? gl : 0));
                int32_t my_code_hi = 0;
                if (LPP == 16 && K >= 16) my_code_hi = __shfl(m_code, src + 1 + (gl + 16 <= K ? gl + 16 : 0));

                float4 vin[V4];
                float4 vo[K + 1][V4];
                const float4* ri = reinterpret_cast<const float4*>(J.tin + (int64_t)(live ? ctx : 0) * D);
#pragma unroll
                for (int i = 0; i < V4; ++i) vin[i] = ri[i * LPP + gl];
#pragma unroll
                for (int k = 0; k <= K; ++k) {
                    const bool ok = live && t[k] >= 0;
                    const float4* ro = reinterpret_cast<const float4*>(J.tout + (int64_t)(ok ? t[k] : 0) * D);
#pragma unroll
                    for (int i = 0; i < V4; ++i)
                        vo[k][i] = ok ? ro[i * LPP + gl] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                }
                double g[K + 1];
                coefficients<K, LPP, V4>(vin, vo, t, lr, live, gl, grp, g, lacc);
                // entries of the out-touches (not the rows touched once)
#pragma unroll
                for (int h = 0; h < (K + LPP) / LPP; ++h) {
                    const int k = gl + h * LPP;
                    double gk = g[0];
                    int32_t tk = t[0];
#pragma unroll
                    for (int jj = 1; jj <= K; ++jj)
                        if (k == jj) {
                            gk = g[jj];
                            tk = t[jj];
                        }
                    if (k <= K && live && tk >= 0 && !((single >> (src + 1 + k)) & 1ull)) {
                        const int32_t code = h == 0 ? my_code : my_code_hi;
                        J.gpos[code & kPosMask] = gk;
                    }
                }
                // out rows touched once: row + g in[ctx] in FP64, rounded once
#pragma unroll
                for (int k = 0; k <= K; ++k) {
                    if (live && t[k] >= 0 && ((single >> (src + 1 + k)) & 1ull)) {
                        float4* dst = reinterpret_cast<float4*>(J.tout + (int64_t)t[k] * D);
#pragma unroll
                        for (int i = 0; i < V4; ++i) {
                            const float4 b = vo[k][i];
                            dst[i * LPP + gl] = make_float4((float)fma(g[k], (double)vin[i].x, (double)b.x),
                                                            (float)fma(g[k], (double)vin[i].y, (double)b.y),
                                                            (float)fma(g[k], (double)vin[i].z, (double)b.z),
                                                            (float)fma(g[k], (double)vin[i].w, (double)b.w));
                        }
                    }
                }
                if (live) {
                    // the context copy is read by the apply of the pair's out
                    // rows touched more than once; an in row touched once is
                    // updated here (its delta rounded to FP32 first, as the
                    // apply rounds the stored delta), others store the delta
                    bool need_ctx = false;
#pragma unroll
                    for (int k = 0; k <= K; ++k)
                        need_ctx = need_ctx || (t[k] >= 0 && !((single >> (src + 1 + k)) & 1ull));
                    const bool in_single = (single >> src) & 1ull;
                    float4* cc = reinterpret_cast<float4*>(J.ctxc + (int64_t)q * D);
                    float4* dp = in_single ? reinterpret_cast<float4*>(J.tin + (int64_t)ctx * D)
                                           : reinterpret_cast<float4*>(J.dinp + (int64_t)pos_in * D);
#pragma unroll
                    for (int i = 0; i < V4; ++i) {
                        if (need_ctx) cc[i * LPP + gl] = vin[i];
                        double ax = 0.0, ay = 0.0, az = 0.0, aw = 0.0;
#pragma unroll
                        for (int k = 0; k <= K; ++k) {
                            ax = fma(g[k], (double)vo[k][i].x, ax);
                            ay = fma(g[k], (double)vo[k][i].y, ay);
                            az = fma(g[k], (double)vo[k][i].z, az);
                            aw = fma(g[k], (double)vo[k][i].w, aw);
                        }
                        float4 dv = make_float4((float)ax, (float)ay, (float)az, (float)aw);
                        if (in_single)
                            dv = make_float4((float)((double)vin[i].x + (double)dv.x),
                                             (float)((double)vin[i].y + (double)dv.y),
                                             (float)((double)vin[i].z + (double)dv.z),
                                             (float)((double)vin[i].w + (double)dv.w));
                        dp[i * LPP + gl] = dv;
                    }
                }
            }
            if (a.njobs > 1) {
                // each job's loss terms to its own partials
                const double l = wave_sum_f64(lacc);
                if (lane == 0) J.loss_part[gw] += l;
                lacc = 0.0;
            }
        }
        if (m < J0.nmb) {
            const uint32_t nseg0 = J0.meta[(int64_t)m * 4];
            if (sidx0 < nseg0 && l16 < pf_seg.z) pf_pair = J0.spair[(int64_t)m * J0.tmax + pf_seg.y + l16];
        }
        if (!grid_sync(a, epoch, clk ? &s_clk[5] : nullptr)) break;
        if (clk) {
            s_clk[6] = wall_clock64();
            s_clk[0] += s_clk[5] - s_clk[4];
            s_clk[1] += s_clk[6] - s_clk[5];
        }

        // ---- apply: one 16-lane group per segment, in and out rows together
        if (m + 1 < J0.nmb) pf_touch = first_touch(m + 1);
        for (int j = 0; j < a.njobs; ++j) {
            const UpdJob& J = a.job[j];
            if (m >= J.nmb) continue;
            const MbDesc dsc = J.desc[m];
            const int32_t* sp = J.spair + (int64_t)m * J.tmax;
            const uint32_t nseg = J.meta[(int64_t)m * 4], nin = J.meta[(int64_t)m * 4 + 1];
            const int4* sg = J.segs + (int64_t)m * J.tmax;
            const double gc = dsc.grid_c;
            for (uint32_t sidx = sidx0; sidx < nseg; sidx += nw * 4) {
                const bool first_seg = j == 0 && sidx == sidx0;
                const int4 sd = first_seg ? pf_seg : sg[sidx];
                const bool out = sidx >= nin;
                const int32_t row = sd.x, start = sd.y, len = sd.z;
                float* table = out ? J.tout : J.tin;
                const float* srcb = out ? J.ctxc : J.dinp;
                float4 cur[AV4];
                const float4* r4 = reinterpret_cast<const float4*>(table + (int64_t)row * D);
#pragma unroll
                for (int i = 0; i < AV4; ++i) cur[i] = r4[i * 16 + l16];
                double acc[D / 16];
#pragma unroll
                for (int e = 0; e < D / 16; ++e) acc[e] = 0.0;
                const bool exact = len > kChunk;
                // touches in batches of 16, one descriptor per lane
                for (int32_t b0 = 0; b0 < len; b0 += 16) {
                    const int32_t nb = min(16, len - b0);
                    // out rows: the touch's coefficient and its pair's context
                    // copy; in rows: the pair's delta at the touch's position
                    double my_g = 1.0;
                    int32_t my_src = start + b0 + l16;
                    if (out && l16 < nb) {
                        my_g = J.gpos[start + b0 + l16];
                        my_src = (first_seg && b0 == 0) ? pf_pair : sp[start + b0 + l16];
                    }
                    for (int32_t i0 = 0; i0 < nb; i0 += kRows) {
                        double gg[kRows];
                        float4 x[kRows][AV4];
#pragma unroll
                        for (int u = 0; u < kRows; ++u) {
                            const bool ok = i0 + u < nb;
                            const int32_t idx = min(i0 + u, 15);
                            gg[u] = __shfl(my_g, (g16 << 4) + idx);
                            const int32_t rr = __shfl(my_src, (g16 << 4) + idx);
                            load_row_if<D, AV4>(x[u], srcb, rr, ok, l16);
                            if (!ok) gg[u] = 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < kRows; ++u) {
                            if (i0 + u >= nb) break;
#pragma unroll
                            for (int i = 0; i < AV4; ++i) {
                                if (exact) {
                                    // order-free: each term rounded onto the grid, sums exact
                                    acc[4 * i + 0] += on_grid(gg[u] * (double)x[u][i].x, gc);
                                    acc[4 * i + 1] += on_grid(gg[u] * (double)x[u][i].y, gc);
                                    acc[4 * i + 2] += on_grid(gg[u] * (double)x[u][i].z, gc);
                                    acc[4 * i + 3] += on_grid(gg[u] * (double)x[u][i].w, gc);
                                } else {
                                    // in rows: g = 1, and 1 * x + acc is exactly x + acc
                                    acc[4 * i + 0] = fma(gg[u], (double)x[u][i].x, acc[4 * i + 0]);
                                    acc[4 * i + 1] = fma(gg[u], (double)x[u][i].y, acc[4 * i + 1]);
                                    acc[4 * i + 2] = fma(gg[u], (double)x[u][i].z, acc[4 * i + 2]);
                                    acc[4 * i + 3] = fma(gg[u], (double)x[u][i].w, acc[4 * i + 3]);
                                }
                            }
                        }
                    }
                }
                float4* d4 = reinterpret_cast<float4*>(table + (int64_t)row * D);
#pragma unroll
                for (int i = 0; i < AV4; ++i) {
                    const float4 c = cur[i];
                    d4[i * 16 + l16] = make_float4((float)((double)c.x + acc[4 * i + 0]),
                                                   (float)((double)c.y + acc[4 * i + 1]),
                                                   (float)((double)c.z + acc[4 * i + 2]),
                                                   (float)((double)c.w + acc[4 * i + 3]));
                }
            }
        }
        if (!grid_sync(a, epoch, clk ? &s_clk[5] : nullptr)) break;
        if (clk) {
            s_clk[2] += s_clk[5] - s_clk[6];
            s_clk[3] += wall_clock64() - s_clk[5];
        }
    }
    if (clk)
        for (int i = 0; i < 4; ++i) atomicAdd(&a.clocks[i], s_clk[i]);
    if (a.njobs == 1) {
        lacc = wave_sum_f64(lacc);
        if (lane == 0) J0.loss_part[gw] += lacc;
    }
}

__global__ void zero_words_kernel(uint32_t* p, int32_t n)
{
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// The forward of the update kernel holds the touches of a wave's pairs in one
// lane each: (64 / lanes per pair) pairs of K + 2 touches must fit 64 lanes
// (K <= 14 at d = 64, where 16 lanes take a pair).
static bool small_touches_fit_wave(int d, int K)
{
    const int pairs_per_wave = d >= 128 ? 2 : 4;
    return pairs_per_wave * (K + 2) <= 64;
}

bool small_path_applies(const Model& m, const felog_train_params& p)
{
    return m.precision == FELOG_PREC_FP32 && m.ctx->sgns_path == 0 &&
           p.minibatch_pairs * (p.negatives + 2) <= kPlanMaxTouches && p.negatives <= 20 &&
           small_touches_fit_wave(m.dim, p.negatives);
}

// Minibatches per plan / update launch pair: the launches' fixed costs spread
// over 64 minibatches are under 1% of their time, and the plans stay small.
int64_t small_minibatches_per_launch() { return 64; }

// Device bytes the small-minibatch update holds for minibatches of P pairs
// and K negatives at dimension d, over a call of B minibatches.
uint64_t small_path_bytes(int64_t P, int K, int d, int64_t B, int num_cus)
{
    const uint64_t T = (uint64_t)(P * (K + 2)), G = (uint64_t)small_minibatches_per_launch();
    const uint64_t blocks = (uint64_t)std::max(kDefaultUpdBlocks, num_cus);
    return 2 * (8 * T * G + 16 * T * G + 4 * T * G + 16 * G) + 8 * T + 2 * 4 * (uint64_t)P * d +
           32 * (uint64_t)std::max<int64_t>(B, 1) + 4 * kFlagStride * (blocks + 2) +
           8 * blocks * (kUpdThreads / 64) + 64;
}

template <int D, int K>
static void* update_kernel_ptr()
{
    return reinterpret_cast<void*>(&sgns_small_update_kernel<D, K>);
}

template <int D>
static void* update_kernel_d(int K)
{
    switch (K) {
#define FELOG_CASE(k) \
    case k: return update_kernel_ptr<D, k>();
        FELOG_CASE(1) FELOG_CASE(2) FELOG_CASE(3) FELOG_CASE(4) FELOG_CASE(5) FELOG_CASE(6)
        FELOG_CASE(7) FELOG_CASE(8) FELOG_CASE(9) FELOG_CASE(10) FELOG_CASE(11) FELOG_CASE(12)
        FELOG_CASE(13) FELOG_CASE(14) FELOG_CASE(15) FELOG_CASE(16) FELOG_CASE(17)
        FELOG_CASE(18) FELOG_CASE(19) FELOG_CASE(20)
#undef FELOG_CASE
        default: fail(FELOG_EUNSUPPORTED, "negatives = %d not supported", K);
    }
}

static void* update_kernel(int D, int K)
{
    if (D == 64) return update_kernel_d<64>(K);
    if (D == 128) return update_kernel_d<128>(K);
    return update_kernel_d<256>(K);
}

static void launch_plan(int K, int nblocks, const PlanBatch& pb, hipStream_t s)
{
    switch (K) {
#define FELOG_CASE(k)                                                                          \
    case k:                                                                                    \
        hipLaunchKernelGGL((sgns_plan_kernel<k>), dim3(nblocks), dim3(kPlanThreads), 0, s, pb); \
        break;
        FELOG_CASE(1) FELOG_CASE(2) FELOG_CASE(3) FELOG_CASE(4) FELOG_CASE(5) FELOG_CASE(6)
        FELOG_CASE(7) FELOG_CASE(8) FELOG_CASE(9) FELOG_CASE(10) FELOG_CASE(11) FELOG_CASE(12)
        FELOG_CASE(13) FELOG_CASE(14) FELOG_CASE(15) FELOG_CASE(16) FELOG_CASE(17)
        FELOG_CASE(18) FELOG_CASE(19) FELOG_CASE(20)
#undef FELOG_CASE
        default: fail(FELOG_EUNSUPPORTED, "negatives = %d not supported", K);
    }
    FELOG_HIP(hipGetLastError());
}

// Model-owned buffers of the persistent path, grown on demand: two sets of
// plan buffers for 64 minibatches (the plans of launch group i + 1 are
// written while the update of group i reads set i mod 2), the out-touch
// coefficients, and each pair's in-row delta and context copy.
static void small_buffers(Model& m, int64_t P, int32_t tmax)
{
    Ctx& c = *m.ctx;
    const int64_t G = small_minibatches_per_launch();
    const int D = m.dim;
    if (m.sm_tmax < tmax || m.sm_G < 2 * G) {
        m.sm_tmax = std::max<int64_t>(m.sm_tmax, tmax);
        m.sm_G = std::max<int64_t>(m.sm_G, 2 * G);
        m.sm_tinfo.alloc(&c, sizeof(int2) * m.sm_tmax * m.sm_G);
        m.sm_segs.alloc(&c, sizeof(int4) * m.sm_tmax * m.sm_G);
        m.sm_meta.alloc(&c, sizeof(uint32_t) * 4 * m.sm_G);
        m.sm_spair.alloc(&c, sizeof(int32_t) * m.sm_tmax * m.sm_G);
        m.sm_gpos.alloc(&c, sizeof(double) * m.sm_tmax);
    }
    if (m.sm_pairs < P || m.sm_dim != D) {
        m.sm_pairs = std::max<int64_t>(m.sm_pairs, P);
        m.sm_dim = D;
        m.sm_dinp.alloc(&c, sizeof(float) * m.sm_pairs * D);
        m.sm_ctxc.alloc(&c, sizeof(float) * m.sm_pairs * D);
    }
}

// Plan arguments of a training call (plan set 0; the caller offsets them).
static PlanArgs plan_args(Model& m, Walks& w, const felog_train_params& p,
                          const int32_t* d_slices, int32_t tmax)
{
    PlanArgs pa{};
    pa.walks = w.data.as<int32_t>();
    pa.W = w.W;
    pa.vcols = w.valid_cols.as<int32_t>();
    pa.slices = d_slices;
    pa.id_base = w.id_base;
    pa.window = p.window;
    pa.seed = p.seed;
    pa.noise = NoiseTable{m.cdf.as<uint64_t>(), m.guide.as<int32_t>(), m.total_weight,
                          m.guide_bits};
    pa.tmax = tmax;
    pa.tinfo = m.sm_tinfo.as<int2>();
    pa.segs = m.sm_segs.as<int4>();
    pa.spair = m.sm_spair.as<int32_t>();
    pa.meta = m.sm_meta.as<uint32_t>();
    pa.row_totals = m.row_totals.as<unsigned long long>();
    return pa;
}

// Descriptors of minibatches [first_mb, end); *last_chunk gets the chunk of
// the last minibatch of each launch group of G, *pairs the pair count.
static std::vector<MbDesc> mb_descs(const Walks& w, const felog_train_params& p,
                                    const TrainSchedule& sch, int64_t first_mb, int64_t end,
                                    int64_t G, std::vector<size_t>* last_chunk, int64_t* pairs)
{
    const int64_t P = p.minibatch_pairs;
    const double lr0 = (double)p.lr_start, lr1 = (double)p.lr_end;
    std::vector<MbDesc> desc((size_t)std::max<int64_t>(1, end - first_mb));
    size_t chunk = 0;
    *pairs = 0;
    for (int64_t b = first_mb; b < end; ++b) {
        while (chunk + 1 < sch.chunk_first_mb.size() && sch.chunk_first_mb[chunk + 1] <= b) ++chunk;
        const int64_t first = (b - sch.chunk_first_mb[chunk]) * P;
        const int64_t np = std::min<int64_t>(P, sch.chunk_pairs[chunk] - first);
        MbDesc& d = desc[(size_t)(b - first_mb)];
        d.vcol_base = sch.chunk_valid_base[chunk];
        d.Wv = (uint32_t)w.chunk_valid[chunk];
        d.first_pair = (uint32_t)first;
        d.npairs = (uint32_t)np;
        const double lr = lr0 - (lr0 - lr1) * (double)b / (double)std::max<int64_t>(1, sch.B - 1);
        d.lr = (float)lr;
        d.grid_c = d.lr > 0.0f ? std::ldexp(1.5, std::ilogb(d.lr) + 17) : 1.5;
        *pairs += np;
        if (last_chunk && ((b - first_mb) % G == G - 1 || b == end - 1)) last_chunk->push_back(chunk);
    }
    return desc;
}

// Workgroups of a persistent update launch: the context's choice (default 64),
// capped at what is resident at once (the launch is cooperative).
int small_update_blocks(const Ctx& c, int D, int K)
{
    int per_cu = 0;
    FELOG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, update_kernel(D, K),
                                                           kUpdThreads, 0));
    FELOG_REQUIRE(per_cu >= 1, "the update kernel does not fit a compute unit");
    const int64_t max_blocks = (int64_t)per_cu * c.num_cus;
    const int64_t want = c.sgns_blocks > 0 ? c.sgns_blocks : kDefaultUpdBlocks;
    return (int)std::max<int64_t>(1, std::min(want, max_blocks));
}

// ------------------------------------------------------- shared launches
// A training call of one model (one job) run inside launches shared with
// other jobs: plans and updates of the jobs' next launch groups together.
// Its plans run on the model's own stream one launch group ahead of the
// shared updates, in two buffer sets (group g uses set g mod 2): the plan of
// group g waits for the update of group g - 2, the update of group g for the
// plan of group g.
struct SmallJob {
    Model* m = nullptr;
    Walks* w = nullptr;
    felog_train_params p{};
    TrainSchedule sch;
    DevBuf slices, ddesc, loss;
    int K = 0, D = 0;
    int32_t tmax = 0;
    int64_t next = 0;        // first minibatch not yet updated
    int64_t planned = 0;     // first minibatch whose plan is not launched
    int64_t end = 0, pairs = 0;
    int nwaves = 0;
    PlanArgs pa{};
    UpdJob uj{};
    hipEvent_t plan_done[2] = {nullptr, nullptr};
    hipEvent_t upd_done[2] = {nullptr, nullptr};
    ~SmallJob()
    {
        for (hipEvent_t e : {plan_done[0], plan_done[1], upd_done[0], upd_done[1]})
            if (e) (void)hipEventDestroy(e);
    }
};

void SmallJobDeleter::operator()(SmallJob* j) const { delete j; }

// Plan arguments of a job's launch group starting at minibatch b (set b / G mod 2).
static PlanArgs group_plan(const SmallJob& j, int64_t b)
{
    const int64_t G = small_minibatches_per_launch();
    const int64_t set = (b / G) & 1;
    PlanArgs pl = j.pa;
    pl.desc = j.ddesc.as<MbDesc>() + b;
    pl.tinfo = j.pa.tinfo + set * G * j.tmax;
    pl.segs = j.pa.segs + set * G * j.tmax;
    pl.spair = j.pa.spair + set * G * j.tmax;
    pl.meta = j.pa.meta + set * G * 4;
    return pl;
}

// Launches the plan of the job's next unplanned launch group on its model's stream.
static void plan_next_group(SmallJob& j)
{
    const int64_t G = small_minibatches_per_launch();
    if (j.planned >= j.end) return;
    const int64_t g = j.planned / G;
    const int set = (int)(g & 1);
    hipStream_t js = j.m->ctx->stream;
    if (g >= 2) FELOG_HIP(hipStreamWaitEvent(js, j.upd_done[set], 0));
    const int nmb = (int)std::min<int64_t>(G, j.end - j.planned);
    PlanBatch pb{};
    pb.job[0] = group_plan(j, j.planned);
    pb.start[0] = 0;
    pb.start[1] = nmb;
    pb.njobs = 1;
    launch_plan(j.K, nmb, pb, js);
    FELOG_HIP(hipEventRecord(j.plan_done[set], js));
    j.planned += nmb;
}

bool small_job_fits(const Model& m, const felog_train_params& p)
{
    return m.precision == FELOG_PREC_FP32 && p.negatives <= 20 &&
           p.minibatch_pairs * (p.negatives + 2) <= kPlanMaxTouches &&
           (m.dim == 64 || m.dim == 128 || m.dim == 256) && small_touches_fit_wave(m.dim, p.negatives);
}

SmallJobPtr small_job_begin(Model& m, Walks& w, const felog_train_params& p, int nblocks)
{
    Ctx& c = *m.ctx;
    FELOG_REQUIRE(small_job_fits(m, p), "the job does not fit the shared persistent update");
    SmallJobPtr j(new SmallJob);
    j->m = &m;
    j->w = &w;
    j->p = p;
    j->sch = train_schedule(w, p);
    j->K = p.negatives;
    j->D = m.dim;
    j->tmax = (int32_t)(p.minibatch_pairs * (p.negatives + 2));
    j->end = j->sch.B;
    j->nwaves = nblocks * (kUpdThreads / 64);
    small_buffers(m, p.minibatch_pairs, j->tmax);
    const std::vector<int32_t> sl = train_slices(w.L, p.window);
    j->slices.alloc(&c, sizeof(int32_t) * std::max<size_t>(sl.size(), 1));
    if (!sl.empty())
        FELOG_HIP(hipMemcpyAsync(j->slices.ptr, sl.data(), sizeof(int32_t) * sl.size(),
                                 hipMemcpyHostToDevice, c.stream));
    const std::vector<MbDesc> desc =
        mb_descs(w, p, j->sch, 0, j->end, small_minibatches_per_launch(), nullptr, &j->pairs);
    j->ddesc.alloc(&c, sizeof(MbDesc) * desc.size());
    FELOG_HIP(hipMemcpyAsync(j->ddesc.ptr, desc.data(), sizeof(MbDesc) * desc.size(),
                             hipMemcpyHostToDevice, c.stream));
    j->loss.alloc(&c, sizeof(double) * j->nwaves);
    FELOG_HIP(hipMemsetAsync(j->loss.ptr, 0, j->loss.bytes, c.stream));
    FELOG_HIP(hipMemsetAsync(m.row_totals.ptr, 0, sizeof(uint64_t) * 3, c.stream));
    j->pa = plan_args(m, w, p, j->slices.as<int32_t>(), j->tmax);
    j->uj.tin = m.tin.as<float>();
    j->uj.tout = m.tout.as<float>();
    j->uj.tmax = j->tmax;
    j->uj.gpos = m.sm_gpos.as<double>();
    j->uj.dinp = m.sm_dinp.as<float>();
    j->uj.ctxc = m.sm_ctxc.as<float>();
    j->uj.loss_part = j->loss.as<double>();
    for (hipEvent_t* e : {&j->plan_done[0], &j->plan_done[1], &j->upd_done[0], &j->upd_done[1]})
        FELOG_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    c.sync();   // the buffers are ready before another stream uses them
    plan_next_group(*j);
    return j;
}

int small_job_dim(const SmallJob& j) { return j.D; }
int small_job_negatives(const SmallJob& j) { return j.K; }
bool small_job_done(const SmallJob& j) { return j.next >= j.end; }

void small_batch_init(SmallBatchCtl& ctl, Ctx& c, int nblocks)
{
    ctl.nblocks = nblocks;
    ctl.epoch = 0;
    ctl.words.alloc(&c, sizeof(uint32_t) * kFlagStride * (nblocks + 2));
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(256), 0, c.stream,
                       ctl.words.as<uint32_t>(), (int32_t)(ctl.words.bytes / sizeof(uint32_t)));
    FELOG_HIP(hipGetLastError());
    c.sync();
}

void small_jobs_step(const std::vector<SmallJob*>& jobs, SmallBatchCtl& ctl, hipStream_t s)
{
    FELOG_REQUIRE(!jobs.empty() && jobs.size() <= (size_t)kMaxBatchJobs,
                  "a shared launch takes 1 to %d jobs", kMaxBatchJobs);
    const int K = jobs[0]->K, D = jobs[0]->D;
    const int64_t G = small_minibatches_per_launch();
    UpdArgs u{};
    int nmb_max = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        SmallJob& j = *jobs[i];
        FELOG_REQUIRE(j.K == K && j.D == D && !small_job_done(j),
                      "jobs of a shared launch need equal d and K and minibatches left");
        FELOG_REQUIRE(j.nwaves == ctl.nblocks * (kUpdThreads / 64),
                      "job prepared for another grid size");
        if (j.planned == j.next) plan_next_group(j);
        const int set = (int)((j.next / G) & 1);
        FELOG_HIP(hipStreamWaitEvent(s, j.plan_done[set], 0));
        const int nmb = (int)std::min<int64_t>(G, j.end - j.next);
        const PlanArgs pl = group_plan(j, j.next);
        UpdJob uj = j.uj;
        uj.desc = pl.desc;
        uj.tinfo = pl.tinfo;
        uj.segs = pl.segs;
        uj.spair = pl.spair;
        uj.meta = pl.meta;
        uj.nmb = nmb;
        u.job[i] = uj;
        nmb_max = std::max(nmb_max, nmb);
    }
    u.njobs = (int32_t)jobs.size();
    u.nmb_max = nmb_max;
    u.flags = ctl.words.as<uint32_t>();
    u.abort = reinterpret_cast<int32_t*>(u.flags + (int64_t)kFlagStride * (ctl.nblocks + 1));
    u.epoch0 = ctl.epoch;
    void* args[] = {&u};
    FELOG_HIP(hipLaunchCooperativeKernel(update_kernel(D, K), dim3(ctl.nblocks), dim3(kUpdThreads),
                                         args, 0, s));
    ctl.epoch += 2u * (uint32_t)nmb_max;
    for (SmallJob* jp : jobs) {
        SmallJob& j = *jp;
        const int set = (int)((j.next / G) & 1);
        FELOG_HIP(hipEventRecord(j.upd_done[set], s));
        j.next += std::min<int64_t>(G, j.end - j.next);
        // the next group's plan beside this update, on the job's stream
        if (j.planned == j.next) plan_next_group(j);
    }
}

bool small_batch_aborted(SmallBatchCtl& ctl, hipStream_t s)
{
    int32_t aborted = 0;
    const int32_t* abort =
        reinterpret_cast<const int32_t*>(ctl.words.as<uint32_t>() + (int64_t)kFlagStride * (ctl.nblocks + 1));
    FELOG_HIP(hipMemcpyAsync(&aborted, abort, sizeof aborted, hipMemcpyDeviceToHost, s));
    FELOG_HIP(hipStreamSynchronize(s));
    return aborted != 0;
}

void small_job_end(SmallJob& j, hipStream_t s, felog_train_stats* stats)
{
    Model& m = *j.m;
    launch_loss_reduce(j.loss.as<double>(), j.nwaves, m.loss_out.as<double>(), s);
    double loss = 0.0;
    unsigned long long rows[3] = {0, 0, 0};
    FELOG_HIP(hipMemcpyAsync(&loss, m.loss_out.ptr, sizeof loss, hipMemcpyDeviceToHost, s));
    FELOG_HIP(hipMemcpyAsync(rows, m.row_totals.ptr, sizeof rows, hipMemcpyDeviceToHost, s));
    FELOG_HIP(hipStreamSynchronize(s));
    if (stats) {
        *stats = felog_train_stats{};
        stats->minibatches = j.end;
        stats->pairs = j.pairs;
        stats->minibatches_total = j.sch.B;
        stats->loss = loss;
        stats->rows_in = (int64_t)rows[0];
        stats->rows_out = (int64_t)rows[1];
        stats->rows_out_single = (int64_t)rows[2];
        stats->path = 1;
    }
}

void train_minibatches_small(Model& m, Walks& w, const felog_train_params& p,
                             const TrainSchedule& sch, const int32_t* d_slices, int64_t first_mb,
                             int64_t end, felog_train_stats* stats)
{
    Ctx& c = *m.ctx;
    const int K = p.negatives;
    const int D = m.dim;
    const int64_t P = p.minibatch_pairs;
    const int32_t tmax = (int32_t)(P * (K + 2));
    FELOG_REQUIRE(tmax <= kPlanMaxTouches, "minibatch of %lld pairs is too large for the "
                  "small-minibatch update", (long long)P);
    FELOG_REQUIRE(D == 64 || D == 128 || D == 256, "dim %d not supported", D);
    const int64_t G = small_minibatches_per_launch();
    void* kern = update_kernel(D, K);
    const int nblocks = small_update_blocks(c, D, K);
    const int nwaves = nblocks * (kUpdThreads / 64);

    small_buffers(m, P, tmax);
    // control words: barrier flags (an unused line, then one per workgroup,
    // each on its own 128-byte line), the abort flag on the next line, then
    // the loss partials, one per wave, and the four phase-clock sums
    const int64_t ctl_words = (int64_t)kFlagStride * (nblocks + 2);
    DevBuf ctl;
    ctl.alloc(&c, sizeof(uint32_t) * ctl_words + sizeof(double) * nwaves +
                      sizeof(unsigned long long) * 4);
    uint32_t* flags = ctl.as<uint32_t>();
    int32_t* abort = reinterpret_cast<int32_t*>(flags + (int64_t)kFlagStride * (nblocks + 1));
    double* loss_part = reinterpret_cast<double*>(flags + ctl_words);
    unsigned long long* clocks = reinterpret_cast<unsigned long long*>(loss_part + nwaves);
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(256), 0, c.stream, flags,
                       (int32_t)(ctl.bytes / sizeof(uint32_t)));
    FELOG_HIP(hipMemsetAsync(m.row_totals.ptr, 0, sizeof(uint64_t) * 3, c.stream));

    const PlanArgs pa = plan_args(m, w, p, d_slices, tmax);

    // every minibatch's descriptor, uploaded once for the call
    std::vector<size_t> last_chunk;   // chunk of the last minibatch of each launch
    int64_t pairs = 0;
    const std::vector<MbDesc> desc = mb_descs(w, p, sch, first_mb, end, G, &last_chunk, &pairs);
    DevBuf ddesc;
    ddesc.alloc(&c, sizeof(MbDesc) * desc.size());
    FELOG_HIP(hipMemcpyAsync(ddesc.ptr, desc.data(), sizeof(MbDesc) * desc.size(),
                             hipMemcpyHostToDevice, c.stream));

    UpdJob uj{};
    uj.tin = m.tin.as<float>();
    uj.tout = m.tout.as<float>();
    uj.tmax = tmax;
    uj.gpos = m.sm_gpos.as<double>();
    uj.dinp = m.sm_dinp.as<float>();
    uj.ctxc = m.sm_ctxc.as<float>();
    uj.loss_part = loss_part;

    // Plans run on the context's second stream one launch group ahead of the
    // updates: plan(i) waits for update(i - 2) (its buffer set), update(i)
    // waits for plan(i).  pipe_ev: [0] start, [1 + set] plan done,
    // [3 + set] update done.
    c.ensure_aux();
    hipStream_t ps = c.aux;
    FELOG_HIP(hipEventRecord(c.pipe_ev[0], c.stream));
    FELOG_HIP(hipStreamWaitEvent(ps, c.pipe_ev[0], 0));
    size_t gated = 0;
    const bool timing = c.timing_every > 0 && !c.timing_pool.empty();
    const size_t tslots = c.timing_pool.size() / 4;
    std::vector<int64_t> slot_nmb(tslots, 0);
    double ms_plan = 0.0, ms_update = 0.0;
    int64_t timed = 0, timed_mb = 0;
    auto harvest = [&](size_t slot) {
        hipEvent_t* e = &c.timing_pool[4 * slot];
        FELOG_HIP(hipEventSynchronize(e[3]));
        float a0 = 0.0f, a1 = 0.0f;
        FELOG_HIP(hipEventElapsedTime(&a0, e[0], e[1]));
        FELOG_HIP(hipEventElapsedTime(&a1, e[2], e[3]));
        ms_plan += a0;
        ms_update += a1;
        ++timed;
        timed_mb += slot_nmb[slot];
        slot_nmb[slot] = 0;
    };
    uint32_t epoch = 0;
    FELOG_HIP(hipEventRecord(c.ev0, c.stream));
    for (int64_t g0 = first_mb, li = 0; g0 < end; g0 += G, ++li) {
        const int64_t g1 = std::min(end, g0 + G);
        const int nmb = (int)(g1 - g0);
        const int set = (int)(li & 1);
        hipEvent_t* e = nullptr;
        if (timing) {
            const size_t slot = (size_t)(li % (int64_t)tslots);
            if (slot_nmb[slot]) harvest(slot);
            slot_nmb[slot] = nmb;
            e = &c.timing_pool[4 * slot];
        }
        // plan of group li, on the second stream
        if (li >= 2) FELOG_HIP(hipStreamWaitEvent(ps, c.pipe_ev[3 + set], 0));
        // the walks of the launch's chunks must be written
        while (gated <= last_chunk[(size_t)li] && gated < w.chunk_ready.size())
            FELOG_HIP(hipStreamWaitEvent(ps, w.chunk_ready[gated++], 0));
        PlanArgs pl = pa;
        pl.desc = ddesc.as<MbDesc>() + (g0 - first_mb);
        pl.tinfo = pa.tinfo + (int64_t)set * G * tmax;
        pl.segs = pa.segs + (int64_t)set * G * tmax;
        pl.spair = pa.spair + (int64_t)set * G * tmax;
        pl.meta = pa.meta + (int64_t)set * G * 4;
        PlanBatch pb{};
        pb.job[0] = pl;
        pb.start[0] = 0;
        pb.start[1] = nmb;
        pb.njobs = 1;
        if (e) FELOG_HIP(hipEventRecord(e[0], ps));
        launch_plan(K, nmb, pb, ps);
        if (e) FELOG_HIP(hipEventRecord(e[1], ps));
        FELOG_HIP(hipEventRecord(c.pipe_ev[1 + set], ps));
        // update of group li, on the context's stream
        FELOG_HIP(hipStreamWaitEvent(c.stream, c.pipe_ev[1 + set], 0));
        UpdArgs u{};
        u.job[0] = uj;
        u.job[0].desc = pl.desc;
        u.job[0].tinfo = pl.tinfo;
        u.job[0].segs = pl.segs;
        u.job[0].spair = pl.spair;
        u.job[0].meta = pl.meta;
        u.job[0].nmb = nmb;
        u.njobs = 1;
        u.nmb_max = nmb;
        u.flags = flags;
        u.abort = abort;
        u.epoch0 = epoch;
        u.clocks = timing ? clocks : nullptr;
        void* args[] = {&u};
        if (e) FELOG_HIP(hipEventRecord(e[2], c.stream));
        FELOG_HIP(hipLaunchCooperativeKernel(kern, dim3(nblocks), dim3(kUpdThreads), args, 0,
                                             c.stream));
        if (e) FELOG_HIP(hipEventRecord(e[3], c.stream));
        FELOG_HIP(hipEventRecord(c.pipe_ev[3 + set], c.stream));
        epoch += 2u * (uint32_t)nmb;
    }
    if (timing)
        for (size_t slot = 0; slot < tslots; ++slot)
            if (slot_nmb[slot]) harvest(slot);
    launch_loss_reduce(loss_part, nwaves, m.loss_out.as<double>(), c.stream);
    FELOG_HIP(hipEventRecord(c.ev1, c.stream));
    double loss = 0.0;
    unsigned long long rows[3] = {0, 0, 0};
    int32_t aborted = 0;
    unsigned long long ticks[4] = {0, 0, 0, 0};
    FELOG_HIP(hipMemcpyAsync(&loss, m.loss_out.ptr, sizeof loss, hipMemcpyDeviceToHost, c.stream));
    FELOG_HIP(hipMemcpyAsync(rows, m.row_totals.ptr, sizeof rows, hipMemcpyDeviceToHost, c.stream));
    FELOG_HIP(hipMemcpyAsync(&aborted, abort, sizeof aborted, hipMemcpyDeviceToHost, c.stream));
    if (timing)
        FELOG_HIP(hipMemcpyAsync(ticks, clocks, sizeof ticks, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    FELOG_HIP(hipStreamSynchronize(ps));
    FELOG_REQUIRE(!aborted, "small-minibatch update: a grid barrier wait exceeded its bound");
    float ms = 0.0f;
    FELOG_HIP(hipEventElapsedTime(&ms, c.ev0, c.ev1));
    if (stats) {
        *stats = felog_train_stats{};
        stats->minibatches = end - first_mb;
        stats->pairs = pairs;
        stats->minibatches_total = sch.B;
        stats->loss = loss;
        stats->ms = ms;
        stats->rows_in = (int64_t)rows[0];
        stats->rows_out = (int64_t)rows[1];
        stats->rows_out_single = (int64_t)rows[2];
        stats->path = 1;
        stats->timed_launches = timed;
        stats->timed_minibatches = timed_mb;
        stats->ms_prep = ms_plan;
        stats->ms_update = ms_update;
        stats->update_blocks = nblocks;
        if (timing && end > first_mb) {
            int khz = 0;   // device wall-clock rate
            FELOG_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c.device));
            const double per = (double)nblocks * (double)(end - first_mb) * (double)khz / 1e3;
            for (int i = 0; i < 4; ++i)
                stats->us_phase[i] = khz > 0 ? (double)ticks[i] / per : 0.0;
        }
    }
}

}  // namespace felog
