// Frequency-aware bitmap compression of a walk corpus (FaBC, Section 5.2.2,
// Eq. (6)-(8)), on the device.
//
// The paper compresses walks on the host to cut their CPU-to-GPU transfer.
// Here walks are generated in HBM, so the codec serves the corpus's trips off
// the device (host fetch, persistence) and back.  Symbols are node ids and -1
// (the padding after an isolated start's only node), so padded positions are
// profiled and compressed like nodes.
//
// Profile: symbol counts (node atomics; padding counted per block), the top
// kFabcMax symbols by (count descending, symbol ascending) through rounds of
// block-local bitonic sorts, then Eq. (8) in one thread: grow k while
// p(k+1) >= c + 0.1 g(k), c = 1/L + 1/32, g(k) = (1 - F_k) + k c, in FP64 with
// every operation rounded as written.
//
// Format (little endian; W walks of L positions, k symbols):
//   header    u32 magic, u32 k, u32 L, u32 0, u64 W, i64 id_base      32 B
//   symbols   i32[k]
//   bitmaps   u8[k][ceil(L/8)][W]: bit j mod 8 of byte j/8 of symbol b's
//             bitmap of walk w is set iff position j of walk w holds symbol b
//   padding   to a multiple of 8 bytes
//   offsets   u64[ceil(W/256)]: residuals before walk 256 i
//   residuals i32[R]: the other positions; per block of 256 walks, position
//             by position, walk ascending
// One thread per walk, 256 walks per block (one offsets entry per block):
// reads of the step-major corpus and the bitmap bytes are coalesced across
// walks, and at each position the block's residuals are compacted with wave
// ballots into consecutive slots, so they are written and read coalesced too.
#include <algorithm>
#include <cstring>

#include "common.h"

namespace felog {

constexpr int kFabcBlock = 256;       // walks per block and per offsets entry
constexpr int kTopSpan = 2048;        // candidates sorted per block
constexpr uint32_t kFabcMagic = 0x43426146u;

struct Cand {
    unsigned long long count;
    int32_t sym;
    int32_t unused;
};

__device__ __forceinline__ bool better(const Cand& a, const Cand& b)
{
    return a.count > b.count || (a.count == b.count && a.sym < b.sym);
}

// ------------------------------------------------------------------ profile
__global__ __launch_bounds__(256) void fabc_count_kernel(const int32_t* __restrict__ data,
                                                         int64_t total,
                                                         unsigned long long* counts,
                                                         unsigned long long* pads)
{
    __shared__ unsigned long long lds[256];
    unsigned long long mine = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * 256) {
        const int32_t v = data[i];
        if (v >= 0) atomicAdd(&counts[v], 1ull);
        else ++mine;
    }
    lds[threadIdx.x] = mine;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && lds[0]) atomicAdd(pads, lds[0]);
}

// One round of the top selection: each block sorts kTopSpan candidates and
// keeps its best kFabcMax.  The first round reads the counts (candidate i is
// symbol i - 1, the padding first), later rounds the previous round's output.
__global__ __launch_bounds__(256) void fabc_top_kernel(const unsigned long long* counts,
                                                       const unsigned long long* pads,
                                                       int64_t n_sym, const Cand* in,
                                                       int64_t n_in, Cand* out)
{
    __shared__ Cand s[kTopSpan];
    const int64_t base = (int64_t)blockIdx.x * kTopSpan;
    const int64_t n = in ? n_in : n_sym + 1;
    for (int e = threadIdx.x; e < kTopSpan; e += 256) {
        const int64_t i = base + e;
        Cand c{0ull, 0x7fffffff, 0};
        if (i < n) {
            if (in) c = in[i];
            else c = Cand{i == 0 ? *pads : counts[i - 1], (int32_t)(i - 1), 0};
        }
        s[e] = c;
    }
    __syncthreads();
    for (int size = 2; size <= kTopSpan; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = threadIdx.x; q < kTopSpan / 2; q += 256) {
                const int i = 2 * q - (q & (stride - 1));
                const int j = i + stride;
                const bool best_first = (i & size) == 0;
                const Cand a = s[i], b = s[j];
                if (best_first ? better(b, a) : better(a, b)) {
                    s[i] = b;
                    s[j] = a;
                }
            }
            __syncthreads();
        }
    if (threadIdx.x < kFabcMax) out[blockIdx.x * kFabcMax + threadIdx.x] = s[threadIdx.x];
}

// Eq. (8) on the ranked candidates (count 0 marks the end of the occurring
// symbols).
__global__ void fabc_select_kernel(const Cand* top, unsigned long long total, int32_t L,
                                   int32_t k_max, int32_t* k_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double c = __dadd_rn(__ddiv_rn(1.0, (double)L), __ddiv_rn(1.0, 32.0));
    double F = 0.0, g = 1.0;
    int32_t k = 0;
    while (k < k_max && top[k].count > 0) {
        const double p = __ddiv_rn((double)top[k].count, (double)total);
        if (!(p >= __dadd_rn(c, __dmul_rn(0.1, g)))) break;
        F = __dadd_rn(F, p);
        ++k;
        g = __dadd_rn(__dsub_rn(1.0, F), __dmul_rn((double)k, c));
    }
    *k_out = k;
}

// -------------------------------------------------------------------- pack
// codes[s + 1] = index of symbol s among the selected ones, or -1.
__global__ void fabc_codes_kernel(int8_t* codes, const int32_t* symbols, int32_t k)
{
    if (threadIdx.x < k) codes[symbols[threadIdx.x] + 1] = (int8_t)threadIdx.x;
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long* lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kFabcBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const unsigned long long t = lds[0];
    __syncthreads();
    return t;
}

// Exclusive scan across the block (Hillis-Steele in LDS).
__device__ __forceinline__ unsigned long long block_excl_u64(unsigned long long v,
                                                             unsigned long long* lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kFabcBlock; off <<= 1) {
        const unsigned long long a = threadIdx.x >= off ? lds[threadIdx.x - off] : 0ull;
        __syncthreads();
        lds[threadIdx.x] += a;
        __syncthreads();
    }
    const unsigned long long r = lds[threadIdx.x] - v;
    __syncthreads();
    return r;
}

// Residuals of each 256-walk block.
__global__ __launch_bounds__(kFabcBlock) void fabc_pack_count_kernel(
    const int32_t* __restrict__ data, int64_t W, int32_t L, const int8_t* __restrict__ codes,
    unsigned long long* block_res)
{
    __shared__ unsigned long long lds[kFabcBlock];
    const int64_t w = (int64_t)blockIdx.x * kFabcBlock + threadIdx.x;
    unsigned long long r = 0;
    if (w < W) {
        // eight positions' loads in flight before their codes are looked up
        for (int32_t j0 = 0; j0 < L; j0 += 8) {
            int32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = j0 + u < L ? data[(int64_t)(j0 + u) * W + w] : 0;
            int8_t c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = codes[v[u] + 1];
#pragma unroll
            for (int u = 0; u < 8; ++u) r += (j0 + u < L && c[u] < 0) ? 1u : 0u;
        }
    }
    const unsigned long long t = block_sum_u64(r, lds);
    if (threadIdx.x == 0) block_res[blockIdx.x] = t;
}

// Exclusive scan of the block residual counts (one block), total in out[nblk].
__global__ __launch_bounds__(kFabcBlock) void fabc_offsets_kernel(
    const unsigned long long* block_res, int64_t nblk, unsigned long long* out)
{
    __shared__ unsigned long long lds[kFabcBlock];
    unsigned long long carry = 0;
    for (int64_t s0 = 0; s0 < nblk; s0 += kFabcBlock) {
        const int64_t i = s0 + threadIdx.x;
        const unsigned long long v = i < nblk ? block_res[i] : 0ull;
        const unsigned long long ex = block_excl_u64(v, lds);
        if (i < nblk) out[i] = carry + ex;
        carry += block_sum_u64(v, lds);
    }
    if (threadIdx.x == 0) out[nblk] = carry;
}

// Slot of this thread's residual among the block's residuals at one position
// (its rank among the lanes and waves below it that hold one), and the
// position's total.  cnt: LDS [2][4], alternating by position, so that one
// barrier per position suffices.
__device__ __forceinline__ uint32_t block_compact(bool res, uint32_t (*cnt)[kFabcBlock / 64],
                                                  int par, uint32_t* total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long m = __ballot(res);
    if (lane == 0) cnt[par][wv] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t below = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kFabcBlock / 64; ++q) {
        const uint32_t c = cnt[par][q];
        below += q < wv ? c : 0u;
        all += c;
    }
    *total = all;
    return below + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

struct PackArgs {
    const int32_t* data;       // step-major [L][W]
    int64_t W;
    int32_t L, k, B8;
    const int8_t* codes;
    uint8_t* bitmaps;          // [k][B8][W]
    const unsigned long long* offsets;
    int32_t* residuals;
};

__global__ __launch_bounds__(kFabcBlock) void fabc_pack_write_kernel(PackArgs a)
{
    __shared__ uint32_t cnt[2][kFabcBlock / 64];
    const int64_t w = (int64_t)blockIdx.x * kFabcBlock + threadIdx.x;
    const bool live = w < a.W;
    unsigned long long at = a.offsets[blockIdx.x];
    for (int32_t j8 = 0; j8 < a.B8; ++j8) {
        uint32_t bytes[kFabcMax];
#pragma unroll
        for (int b = 0; b < kFabcMax; ++b) bytes[b] = 0u;
        // the group's eight loads and code lookups first, then its compactions
        int32_t v[8];
        int c[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int32_t j = 8 * j8 + t;
            v[t] = live && j < a.L ? a.data[(int64_t)j * a.W + w] : 0;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) c[t] = live ? a.codes[v[t] + 1] : 0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int32_t j = 8 * j8 + t;
            if (j >= a.L) break;                 // uniform across the block
            uint32_t total;
            const uint32_t slot = block_compact(live && c[t] < 0, cnt, j & 1, &total);
            if (live && c[t] < 0) a.residuals[at + slot] = v[t];
            at += total;
#pragma unroll
            for (int b = 0; b < kFabcMax; ++b) bytes[b] |= (c[t] == b ? 1u : 0u) << t;
        }
        if (live) {
#pragma unroll
            for (int b = 0; b < kFabcMax; ++b)
                if (b < a.k) a.bitmaps[((int64_t)b * a.B8 + j8) * a.W + w] = (uint8_t)bytes[b];
        }
    }
}

// ------------------------------------------------------------------ unpack
// Error bits: 1 overlapping or stray bitmap bits, 2 offsets that disagree with
// the bitmaps, 4 residuals past the end, 8 a residual outside [-1, n).
struct UnpackArgs {
    int64_t W;
    int32_t L, k, B8;
    int32_t n;                 // nodes of the graph
    const int32_t* symbols;
    const uint8_t* bitmaps;
    const unsigned long long* offsets;
    const int32_t* residuals;
    unsigned long long R;
    int32_t* data;             // step-major [L][W]
    uint32_t* err;
};

__global__ __launch_bounds__(kFabcBlock) void fabc_unpack_kernel(UnpackArgs a)
{
    __shared__ uint32_t cnt[2][kFabcBlock / 64];
    const int64_t w = (int64_t)blockIdx.x * kFabcBlock + threadIdx.x;
    const bool live = w < a.W;
    const int64_t nblk = (a.W + kFabcBlock - 1) / kFabcBlock;
    const unsigned long long first = a.offsets[blockIdx.x];
    const unsigned long long next = blockIdx.x + 1 < nblk ? a.offsets[blockIdx.x + 1] : a.R;
    uint32_t bad = 0;
    unsigned long long at = first;
    for (int32_t j8 = 0; j8 < a.B8; ++j8) {
        uint32_t by[kFabcMax];
        uint32_t any = 0, sum = 0;
#pragma unroll
        for (int b = 0; b < kFabcMax; ++b) {
            by[b] = live && b < a.k ? a.bitmaps[((int64_t)b * a.B8 + j8) * a.W + w] : 0u;
            any |= by[b];
            sum += __popc(by[b]);
        }
        const int32_t valid = min(8, a.L - 8 * j8);
        if (sum != (uint32_t)__popc(any) || (any >> valid) != 0u) bad |= 1u;
        // the group's eight compactions first, then its residual loads together
        int hit[8];
        unsigned long long idx[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int32_t j = 8 * j8 + t;
            hit[t] = -1;
            idx[t] = 0;
            if (j >= a.L) break;                 // uniform across the block
#pragma unroll
            for (int b = 0; b < kFabcMax; ++b)
                if (hit[t] < 0 && ((by[b] >> t) & 1u)) hit[t] = b;
            uint32_t total;
            idx[t] = at + block_compact(live && hit[t] < 0, cnt, j & 1, &total);
            at += total;
        }
        int32_t v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            v[t] = -1;
            if (!live || 8 * j8 + t >= a.L) continue;
            if (hit[t] >= 0) {
                v[t] = a.symbols[hit[t]];
            } else if (idx[t] < a.R) {
                v[t] = a.residuals[idx[t]];
                if (v[t] < -1 || v[t] >= a.n) {
                    bad |= 8u;
                    v[t] = -1;
                }
            } else {
                bad |= 4u;
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (live && 8 * j8 + t < a.L) a.data[(int64_t)(8 * j8 + t) * a.W + w] = v[t];
    }
    if (threadIdx.x == 0 && at != next) bad |= 2u;
    if (bad) atomicOr(a.err, bad);
}

// -------------------------------------------------------------------- host
static int64_t packed_fixed_bytes(int64_t W, int32_t L, int32_t k)
{
    int64_t used = 32 + 4 * (int64_t)k + (int64_t)k * ((L + 7) / 8) * W;
    used += (8 - used % 8) % 8;
    return used + 8 * ((W + kFabcBlock - 1) / kFabcBlock);
}

static void region_offsets(const Packed& p, int64_t* bitmaps, int64_t* offsets, int64_t* res)
{
    *bitmaps = 32 + 4 * (int64_t)p.k;
    int64_t used = *bitmaps + (int64_t)p.k * ((p.L + 7) / 8) * p.W;
    used += (8 - used % 8) % 8;
    *offsets = used;
    *res = used + 8 * ((p.W + kFabcBlock - 1) / kFabcBlock);
}

void fabc_profile(const Walks& w, int32_t k_max, int32_t* k, int32_t* symbols,
                  uint64_t* counts, int32_t* n_ranked, uint64_t* total)
{
    Ctx& c = *w.g->ctx;
    c.make_current();
    const int64_t n = w.g->n;
    const int64_t positions = w.W * (int64_t)w.L;
    DevBuf cnt, pads, top_a, top_b, kbuf;
    cnt.alloc(&c, sizeof(unsigned long long) * std::max<int64_t>(n, 1));
    pads.alloc(&c, sizeof(unsigned long long));
    FELOG_HIP(hipMemsetAsync(cnt.ptr, 0, cnt.bytes, c.stream));
    FELOG_HIP(hipMemsetAsync(pads.ptr, 0, pads.bytes, c.stream));
    if (positions > 0) {
        const int64_t blocks = std::min<int64_t>((positions + 255) / 256, (int64_t)c.num_cus * 16);
        hipLaunchKernelGGL(fabc_count_kernel, dim3(blocks), dim3(256), 0, c.stream,
                           w.data.as<int32_t>(), positions, cnt.as<unsigned long long>(),
                           pads.as<unsigned long long>());
    }
    int64_t n_cand = n + 1;
    int64_t nb = (n_cand + kTopSpan - 1) / kTopSpan;
    top_a.alloc(&c, sizeof(Cand) * nb * kFabcMax);
    top_b.alloc(&c, sizeof(Cand) * std::max<int64_t>((nb * kFabcMax + kTopSpan - 1) / kTopSpan, 1) *
                        kFabcMax);
    hipLaunchKernelGGL(fabc_top_kernel, dim3(nb), dim3(256), 0, c.stream,
                       cnt.as<unsigned long long>(), pads.as<unsigned long long>(), n,
                       (const Cand*)nullptr, (int64_t)0, top_a.as<Cand>());
    Cand* cur = top_a.as<Cand>();
    Cand* nxt = top_b.as<Cand>();
    n_cand = nb * kFabcMax;
    while (nb > 1) {
        nb = (n_cand + kTopSpan - 1) / kTopSpan;
        hipLaunchKernelGGL(fabc_top_kernel, dim3(nb), dim3(256), 0, c.stream,
                           (const unsigned long long*)nullptr,
                           (const unsigned long long*)nullptr, (int64_t)0, cur, n_cand, nxt);
        std::swap(cur, nxt);
        n_cand = nb * kFabcMax;
    }
    kbuf.alloc(&c, sizeof(int32_t));
    hipLaunchKernelGGL(fabc_select_kernel, dim3(1), dim3(64), 0, c.stream, cur,
                       (unsigned long long)positions, w.L, std::min(k_max, kFabcMax),
                       kbuf.as<int32_t>());
    FELOG_HIP(hipGetLastError());
    Cand top[kFabcMax];
    int32_t kk = 0;
    FELOG_HIP(hipMemcpyAsync(top, cur, sizeof top, hipMemcpyDeviceToHost, c.stream));
    FELOG_HIP(hipMemcpyAsync(&kk, kbuf.ptr, sizeof kk, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    int32_t m = 0;
    for (int i = 0; i < kFabcMax && i < k_max && top[i].count > 0; ++i) {
        symbols[i] = top[i].sym;
        counts[i] = top[i].count;
        ++m;
    }
    *k = kk;
    *n_ranked = m;
    *total = (uint64_t)positions;
}

void fabc_pack(const Walks& w, int32_t k, const int32_t* symbols, Packed& p, double* ms)
{
    Ctx& c = *w.g->ctx;
    c.make_current();
    const int64_t n = w.g->n, W = w.W;
    const int32_t L = w.L;
    const int64_t nblk = (W + kFabcBlock - 1) / kFabcBlock;
    DevBuf codes, syms, block_res, offs;
    codes.alloc(&c, (size_t)n + 1);
    syms.alloc(&c, sizeof(int32_t) * kFabcMax);
    block_res.alloc(&c, sizeof(unsigned long long) * std::max<int64_t>(nblk, 1));
    offs.alloc(&c, sizeof(unsigned long long) * (nblk + 1));
    FELOG_HIP(hipMemsetAsync(codes.ptr, 0xff, codes.bytes, c.stream));
    if (k > 0)
        FELOG_HIP(hipMemcpyAsync(syms.ptr, symbols, sizeof(int32_t) * k, hipMemcpyHostToDevice,
                                 c.stream));
    FELOG_HIP(hipEventRecord(c.ev0, c.stream));
    hipLaunchKernelGGL(fabc_codes_kernel, dim3(1), dim3(64), 0, c.stream, codes.as<int8_t>(),
                       syms.as<int32_t>(), k);
    if (nblk > 0)
        hipLaunchKernelGGL(fabc_pack_count_kernel, dim3(nblk), dim3(kFabcBlock), 0, c.stream,
                           w.data.as<int32_t>(), W, L, codes.as<int8_t>(),
                           block_res.as<unsigned long long>());
    hipLaunchKernelGGL(fabc_offsets_kernel, dim3(1), dim3(kFabcBlock), 0, c.stream,
                       block_res.as<unsigned long long>(), nblk, offs.as<unsigned long long>());
    FELOG_HIP(hipEventRecord(c.ev1, c.stream));
    unsigned long long R = 0;
    FELOG_HIP(hipMemcpyAsync(&R, offs.as<unsigned long long>() + nblk, sizeof R,
                             hipMemcpyDeviceToHost, c.stream));
    c.sync();
    float ms_count = 0.0f;
    FELOG_HIP(hipEventElapsedTime(&ms_count, c.ev0, c.ev1));

    p.g = w.g;
    p.k = k;
    p.L = L;
    p.W = W;
    p.id_base = w.id_base;
    p.R = (int64_t)R;
    for (int b = 0; b < k; ++b) p.symbols[b] = symbols[b];
    p.bytes = packed_fixed_bytes(W, L, k) + 4 * p.R;
    p.buf.alloc(&c, (size_t)p.bytes);
    int64_t o_bm, o_off, o_res;
    region_offsets(p, &o_bm, &o_off, &o_res);
    std::vector<uint8_t> head(o_bm, 0);
    const uint32_t h32[4] = {kFabcMagic, (uint32_t)k, (uint32_t)L, 0u};
    std::memcpy(head.data(), h32, 16);
    std::memcpy(head.data() + 16, &W, 8);
    std::memcpy(head.data() + 24, &w.id_base, 8);
    if (k > 0) std::memcpy(head.data() + 32, symbols, 4 * (size_t)k);
    uint8_t* base = p.buf.as<uint8_t>();
    FELOG_HIP(hipMemcpyAsync(base, head.data(), head.size(), hipMemcpyHostToDevice, c.stream));
    const int64_t bm_end = o_bm + (int64_t)k * ((L + 7) / 8) * W;
    if (o_off > bm_end) FELOG_HIP(hipMemsetAsync(base + bm_end, 0, o_off - bm_end, c.stream));
    if (nblk > 0)
        FELOG_HIP(hipMemcpyAsync(base + o_off, offs.ptr, 8 * (size_t)nblk,
                                 hipMemcpyDeviceToDevice, c.stream));
    FELOG_HIP(hipEventRecord(c.ev0, c.stream));
    if (nblk > 0) {
        PackArgs a{w.data.as<int32_t>(), W, L, k, (L + 7) / 8, codes.as<int8_t>(), base + o_bm,
                   reinterpret_cast<const unsigned long long*>(base + o_off),
                   reinterpret_cast<int32_t*>(base + o_res)};
        hipLaunchKernelGGL(fabc_pack_write_kernel, dim3(nblk), dim3(kFabcBlock), 0, c.stream, a);
    }
    FELOG_HIP(hipGetLastError());
    FELOG_HIP(hipEventRecord(c.ev1, c.stream));
    c.sync();
    float ms_write = 0.0f;
    FELOG_HIP(hipEventElapsedTime(&ms_write, c.ev0, c.ev1));
    if (ms) {
        ms[0] = ms_count;
        ms[1] = ms_write;
    }
}

void fabc_from_host(Graph& g, const void* host, int64_t bytes, Packed& p)
{
    Ctx& c = *g.ctx;
    c.make_current();
    FELOG_REQUIRE(bytes >= 32, "a packed corpus has a 32-byte header; got %lld bytes",
                  (long long)bytes);
    uint32_t h32[4];
    int64_t W, id_base;
    std::memcpy(h32, host, 16);
    std::memcpy(&W, (const uint8_t*)host + 16, 8);
    std::memcpy(&id_base, (const uint8_t*)host + 24, 8);
    FELOG_REQUIRE(h32[0] == kFabcMagic && h32[3] == 0u, "not a packed walk corpus");
    const int32_t k = (int32_t)h32[1], L = (int32_t)h32[2];
    FELOG_REQUIRE(k >= 0 && k <= kFabcMax && L >= 1 && W >= 0,
                  "packed header out of range (k %d, L %d, W %lld)", k, L, (long long)W);
    FELOG_REQUIRE(W <= (int64_t)1 << 40 && (int64_t)L * W <= (int64_t)1 << 42,
                  "packed corpus too large (W %lld, L %d)", (long long)W, L);
    const int64_t fixed = packed_fixed_bytes(W, L, k);
    FELOG_REQUIRE(bytes >= fixed && (bytes - fixed) % 4 == 0 &&
                      (bytes - fixed) / 4 <= (int64_t)L * W,
                  "packed corpus of %lld bytes does not fit its header", (long long)bytes);
    const int32_t* syms = reinterpret_cast<const int32_t*>((const uint8_t*)host + 32);
    for (int b = 0; b < k; ++b) {
        int32_t s;
        std::memcpy(&s, syms + b, 4);
        FELOG_REQUIRE(s >= -1 && s < g.n, "packed symbol %d outside [-1, %d)", s, g.n);
        for (int q = 0; q < b; ++q) FELOG_REQUIRE(p.symbols[q] != s, "packed symbol %d repeated", s);
        p.symbols[b] = s;
    }
    p.g = &g;
    p.k = k;
    p.L = L;
    p.W = W;
    p.id_base = id_base;
    p.R = (bytes - fixed) / 4;
    p.bytes = bytes;
    p.buf.alloc(&c, (size_t)bytes);
    FELOG_HIP(hipMemcpyAsync(p.buf.ptr, host, (size_t)bytes, hipMemcpyHostToDevice, c.stream));
    c.sync();
}

void fabc_unpack(const Packed& p, Walks& w, double* ms)
{
    Ctx& c = *p.g->ctx;
    c.make_current();
    w.g = p.g;
    w.W = p.W;
    w.L = p.L;
    w.id_base = p.id_base;
    w.data.alloc(&c, sizeof(int32_t) * std::max<int64_t>(p.W * p.L, 1));
    DevBuf err;
    err.alloc(&c, sizeof(uint32_t));
    FELOG_HIP(hipMemsetAsync(err.ptr, 0, sizeof(uint32_t), c.stream));
    int64_t o_bm, o_off, o_res;
    region_offsets(p, &o_bm, &o_off, &o_res);
    const uint8_t* base = p.buf.as<uint8_t>();
    const int64_t nblk = (p.W + kFabcBlock - 1) / kFabcBlock;
    FELOG_HIP(hipEventRecord(c.ev0, c.stream));
    if (nblk > 0) {
        UnpackArgs a{p.W, p.L, p.k, (p.L + 7) / 8, p.g->n,
                     reinterpret_cast<const int32_t*>(base + 32), base + o_bm,
                     reinterpret_cast<const unsigned long long*>(base + o_off),
                     reinterpret_cast<const int32_t*>(base + o_res),
                     (unsigned long long)p.R, w.data.as<int32_t>(), err.as<uint32_t>()};
        hipLaunchKernelGGL(fabc_unpack_kernel, dim3(nblk), dim3(kFabcBlock), 0, c.stream, a);
    }
    FELOG_HIP(hipGetLastError());
    FELOG_HIP(hipEventRecord(c.ev1, c.stream));
    uint32_t bad = 0;
    FELOG_HIP(hipMemcpyAsync(&bad, err.ptr, sizeof bad, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    float t = 0.0f;
    FELOG_HIP(hipEventElapsedTime(&t, c.ev0, c.ev1));
    if (ms) *ms = t;
    FELOG_REQUIRE(bad == 0u, "corrupt packed corpus (%s%s%s%s)",
                  (bad & 1u) ? "overlapping or stray bitmap bits " : "",
                  (bad & 2u) ? "offsets disagree with the bitmaps " : "",
                  (bad & 4u) ? "residuals missing " : "",
                  (bad & 8u) ? "residual outside [-1, n) " : "");
}

}  // namespace felog
