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
// The pack and unpack launches give one wave to each 256-walk block of the
// format and four consecutive walks to each lane, so corpus rows and bitmap
// bytes are read and written 16 and 4 bytes per lane, and at each position the
// block's residuals are compacted with four wave ballots into consecutive
// slots (coalesced, and no barrier).
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
// The selected symbols, by value (k of them, the rest unused).
struct Symbols {
    int32_t s[kFabcMax];
};

// Index of v among the k selected symbols, or -1: compares against registers
// (a table lookup per position would be a random access per lane).
__device__ __forceinline__ int symbol_code(int32_t v, const Symbols& sy, int32_t k)
{
    int c = -1;
    for (int b = k - 1; b >= 0; --b)
        if (v == sy.s[b]) c = b;
    return c;
}

constexpr int kWalksPerLane = 4;

__device__ __forceinline__ void load4(const int32_t* row, int64_t w0, int64_t W, bool vec,
                                      int32_t (&v)[kWalksPerLane])
{
    if (vec && w0 + 3 < W) {
        const int4 q = *reinterpret_cast<const int4*>(row + w0);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
#pragma unroll
        for (int i = 0; i < kWalksPerLane; ++i) v[i] = w0 + i < W ? row[w0 + i] : 0;
    }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Slots of the lane's flagged walks among the wave's flagged walks at one
// position (walk order), and their total.
__device__ __forceinline__ void wave_slots(const bool (&f)[kWalksPerLane],
                                           uint32_t (&slot)[kWalksPerLane], uint32_t* total)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t below = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kWalksPerLane; ++i) {
        const unsigned long long m = __ballot(f[i]);
        below += (uint32_t)__popcll(m & lt);
        all += (uint32_t)__popcll(m);
    }
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < kWalksPerLane; ++i) {
        slot[i] = below + mine;
        mine += f[i] ? 1u : 0u;
    }
    *total = all;
}

// Stores with the nontemporal hint: the unpacked corpus is written once and
// not read again by the launch (2.47 -> 2.35 ms for the R-MAT 2^20 round-1
// corpus; on the packing side's scattered stores the hint was slower).
typedef int nt_i4x __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_nt4(int32_t* p, int32_t a, int32_t b, int32_t c, int32_t d)
{
    __builtin_nontemporal_store(nt_i4x{a, b, c, d}, reinterpret_cast<nt_i4x*>(p));
}

// Bit t of x moved to bit 4t (x < 256).
__device__ __forceinline__ uint32_t spread_nibbles(uint32_t x)
{
    x = (x | (x << 12)) & 0x000F000Fu;
    x = (x | (x << 6)) & 0x03030303u;
    x = (x | (x << 3)) & 0x11111111u;
    return x;
}

// Residuals of each 256-walk block (one wave per block).
__global__ __launch_bounds__(256) void fabc_pack_count_kernel(
    const int32_t* __restrict__ data, int64_t W, int32_t L, Symbols sy, int32_t k,
    unsigned long long* block_res, int64_t nblk)
{
    const int64_t fb = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (fb >= nblk) return;
    const int64_t w0 = fb * kFabcBlock + (threadIdx.x & 63) * kWalksPerLane;
    const bool vec = (W & 3) == 0;
    unsigned long long r = 0;
    for (int32_t j = 0; j < L; ++j) {
        int32_t v[kWalksPerLane];
        load4(data + (int64_t)j * W, w0, W, vec, v);
#pragma unroll
        for (int i = 0; i < kWalksPerLane; ++i)
            r += (w0 + i < W && symbol_code(v[i], sy, k) < 0) ? 1u : 0u;
    }
    r = wave_sum_u64(r);
    if ((threadIdx.x & 63) == 0) block_res[fb] = r;
}

// Exclusive scan of the block residual counts in one block of 1024 threads,
// total in out[nblk]: each thread sums a contiguous run, the runs' sums are
// scanned through wave shuffles and LDS, and each thread writes its run.
constexpr int kOffsetsThreads = 1024;

__global__ __launch_bounds__(kOffsetsThreads) void fabc_offsets_kernel(
    const unsigned long long* block_res, int64_t nblk, unsigned long long* out)
{
    __shared__ unsigned long long wsum[kOffsetsThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t per = (nblk + kOffsetsThreads - 1) / kOffsetsThreads;
    const int64_t b = (int64_t)threadIdx.x * per, e = min(nblk, b + per);
    unsigned long long run = 0;
#pragma unroll 8
    for (int64_t i = b; i < e; ++i) run += block_res[i];
    unsigned long long incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long x = __shfl_up(incl, off);
        if (lane >= off) incl += x;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    unsigned long long before = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kOffsetsThreads / 64; ++q) {
        before += q < wv ? wsum[q] : 0ull;
        total += wsum[q];
    }
    unsigned long long at = before + incl - run;
    for (int64_t i = b; i < e; ++i) {
        out[i] = at;
        at += block_res[i];
    }
    if (threadIdx.x == 0) out[nblk] = total;
}

struct PackArgs {
    const int32_t* data;       // step-major [L][W]
    int64_t W, nblk;
    int32_t L, k, B8;
    Symbols sy;
    uint8_t* bitmaps;          // [k][B8][W]
    const unsigned long long* offsets;
    int32_t* residuals;
};

__global__ __launch_bounds__(256) void fabc_pack_write_kernel(PackArgs a)
{
    const int64_t fb = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (fb >= a.nblk) return;
    const int64_t w0 = fb * kFabcBlock + (threadIdx.x & 63) * kWalksPerLane;
    const bool vec = (a.W & 3) == 0;
    const bool full = w0 + kWalksPerLane - 1 < a.W;
    unsigned long long at = a.offsets[fb];
    for (int32_t j8 = 0; j8 < a.B8; ++j8) {
        // bit t of hm[i]: position 8 j8 + t of walk i holds a selected symbol,
        // whose index is nibble t of cw[i]
        uint32_t cw[kWalksPerLane] = {0u, 0u, 0u, 0u}, hm[kWalksPerLane] = {0u, 0u, 0u, 0u};
        for (int t = 0; t < 8; ++t) {
            const int32_t j = 8 * j8 + t;
            if (j >= a.L) break;
            int32_t v[kWalksPerLane];
            load4(a.data + (int64_t)j * a.W, w0, a.W, vec, v);
            bool f[kWalksPerLane];
#pragma unroll
            for (int i = 0; i < kWalksPerLane; ++i) {
                const int c = symbol_code(v[i], a.sy, a.k);
                f[i] = w0 + i < a.W && c < 0;
                cw[i] |= (uint32_t)(c < 0 ? 0 : c) << (4 * t);
                hm[i] |= (c >= 0 ? 1u : 0u) << t;
            }
            uint32_t slot[kWalksPerLane], total;
            wave_slots(f, slot, &total);
#pragma unroll
            for (int i = 0; i < kWalksPerLane; ++i)
                if (f[i]) a.residuals[at + slot[i]] = v[i];
            at += total;
        }
        for (int32_t b = 0; b < a.k; ++b) {
            uint32_t q = 0;
#pragma unroll
            for (int i = 0; i < kWalksPerLane; ++i) {
                uint32_t by = 0;
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    by |= (((hm[i] >> t) & 1u) && ((cw[i] >> (4 * t)) & 15u) == (uint32_t)b ? 1u
                                                                                          : 0u)
                          << t;
                q |= by << (8 * i);
            }
            uint8_t* dst = a.bitmaps + ((int64_t)b * a.B8 + j8) * a.W + w0;
            if (vec && full) {
                *reinterpret_cast<uint32_t*>(dst) = q;
            } else {
#pragma unroll
                for (int i = 0; i < kWalksPerLane; ++i)
                    if (w0 + i < a.W) dst[i] = (uint8_t)(q >> (8 * i));
            }
        }
    }
}

// ------------------------------------------------------------------ unpack
// Error bits: 1 overlapping or stray bitmap bits, 2 offsets that disagree with
// the bitmaps, 4 residuals past the end, 8 a residual outside [-1, n).
struct UnpackArgs {
    int64_t W, nblk;
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

__global__ __launch_bounds__(256) void fabc_unpack_kernel(UnpackArgs a)
{
    const int64_t fb = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (fb >= a.nblk) return;
    const int64_t w0 = fb * kFabcBlock + (threadIdx.x & 63) * kWalksPerLane;
    const bool vec = (a.W & 3) == 0;
    const bool full = w0 + kWalksPerLane - 1 < a.W;
    const unsigned long long next = fb + 1 < a.nblk ? a.offsets[fb + 1] : a.R;
    unsigned long long at = a.offsets[fb];
    uint32_t bad = 0;
    for (int32_t j8 = 0; j8 < a.B8; ++j8) {
        // nibble t of cw[i]: the symbol index at position 8 j8 + t of walk i where
        // bit t of any[i] is set
        uint32_t cw[kWalksPerLane] = {0u, 0u, 0u, 0u};
        uint32_t any[kWalksPerLane] = {0u, 0u, 0u, 0u}, sum[kWalksPerLane] = {0u, 0u, 0u, 0u};
        for (int32_t b = 0; b < a.k; ++b) {
            const uint8_t* src = a.bitmaps + ((int64_t)b * a.B8 + j8) * a.W + w0;
            uint32_t q = 0;
            if (vec && full) {
                q = *reinterpret_cast<const uint32_t*>(src);
            } else {
#pragma unroll
                for (int i = 0; i < kWalksPerLane; ++i)
                    if (w0 + i < a.W) q |= (uint32_t)src[i] << (8 * i);
            }
#pragma unroll
            for (int i = 0; i < kWalksPerLane; ++i) {
                const uint32_t by = (q >> (8 * i)) & 255u;
                any[i] |= by;
                sum[i] += __popc(by);
                cw[i] |= spread_nibbles(by) * (uint32_t)b;
            }
        }
        const int32_t valid = min(8, a.L - 8 * j8);
#pragma unroll
        for (int i = 0; i < kWalksPerLane; ++i)
            if (sum[i] != (uint32_t)__popc(any[i]) || (any[i] >> valid) != 0u) bad |= 1u;
        // the group's eight positions: slots and reads first (the residual
        // offsets follow from the bitmaps alone, so all reads are in flight
        // together), then the checks and the stores
        int32_t v[8][kWalksPerLane];
        uint32_t from_res = 0;   // bit 4 t + i: v[t][i] was read from the residuals
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t >= valid) break;
            int hit[kWalksPerLane];
            bool f[kWalksPerLane];
#pragma unroll
            for (int i = 0; i < kWalksPerLane; ++i) {
                hit[i] = ((any[i] >> t) & 1u) ? (int)((cw[i] >> (4 * t)) & 15u) : -1;
                f[i] = w0 + i < a.W && hit[i] < 0;
            }
            uint32_t slot[kWalksPerLane], total;
            wave_slots(f, slot, &total);
#pragma unroll
            for (int i = 0; i < kWalksPerLane; ++i) {
                v[t][i] = -1;
                if (hit[i] >= 0 && hit[i] < a.k) {
                    v[t][i] = a.symbols[hit[i]];
                } else if (f[i]) {
                    if (at + slot[i] < a.R) {
                        v[t][i] = a.residuals[at + slot[i]];
                        from_res |= 1u << (4 * t + i);
                    } else {
                        bad |= 4u;
                    }
                }
            }
            at += total;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t >= valid) break;
#pragma unroll
            for (int i = 0; i < kWalksPerLane; ++i)
                if (((from_res >> (4 * t + i)) & 1u) && (v[t][i] < -1 || v[t][i] >= a.n)) {
                    bad |= 8u;
                    v[t][i] = -1;
                }
            int32_t* row = a.data + (int64_t)(8 * j8 + t) * a.W;
            if (vec && full) {
                store_nt4(row + w0, v[t][0], v[t][1], v[t][2], v[t][3]);
            } else {
#pragma unroll
                for (int i = 0; i < kWalksPerLane; ++i)
                    if (w0 + i < a.W) row[w0 + i] = v[t][i];
            }
        }
    }
    if ((threadIdx.x & 63) == 0 && at != next) bad |= 2u;
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
    const int64_t W = w.W;
    const int32_t L = w.L;
    const int64_t nblk = (W + kFabcBlock - 1) / kFabcBlock;
    DevBuf block_res, offs;
    Symbols sy{};
    for (int b = 0; b < k; ++b) sy.s[b] = symbols[b];
    block_res.alloc(&c, sizeof(unsigned long long) * std::max<int64_t>(nblk, 1));
    offs.alloc(&c, sizeof(unsigned long long) * (nblk + 1));
    FELOG_HIP(hipEventRecord(c.ev0, c.stream));
    if (nblk > 0)
        hipLaunchKernelGGL(fabc_pack_count_kernel, dim3((nblk + 3) / 4), dim3(256), 0, c.stream,
                           w.data.as<int32_t>(), W, L, sy, k, block_res.as<unsigned long long>(),
                           nblk);
    hipLaunchKernelGGL(fabc_offsets_kernel, dim3(1), dim3(kOffsetsThreads), 0, c.stream,
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
        PackArgs a{w.data.as<int32_t>(), W, nblk, L, k, (L + 7) / 8, sy, base + o_bm,
                   reinterpret_cast<const unsigned long long*>(base + o_off),
                   reinterpret_cast<int32_t*>(base + o_res)};
        hipLaunchKernelGGL(fabc_pack_write_kernel, dim3((nblk + 3) / 4), dim3(256), 0, c.stream,
                           a);
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
        UnpackArgs a{p.W, nblk, p.L, p.k, (p.L + 7) / 8, p.g->n,
                     reinterpret_cast<const int32_t*>(base + 32), base + o_bm,
                     reinterpret_cast<const unsigned long long*>(base + o_off),
                     reinterpret_cast<const int32_t*>(base + o_res),
                     (unsigned long long)p.R, w.data.as<int32_t>(), err.as<uint32_t>()};
        hipLaunchKernelGGL(fabc_unpack_kernel, dim3((nblk + 3) / 4), dim3(256), 0, c.stream, a);
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
