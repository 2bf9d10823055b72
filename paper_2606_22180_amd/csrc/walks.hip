// Graph checks and random-walk generation (Sample of Algorithm 1).
//
// Uniform walks follow the DeepWalk sampler of Section 2 ("Sampling
// process"): each transition picks a neighbour of the current node
// uniformly.  node2vec walks (named in Sections 3 and 5.4) bias the choice by
// the previous node with return parameter p and in-out parameter q; they are
// drawn by rejection so no per-edge alias tables are needed.
//
// Layout: walks are stored step-major, walk[t][col] at t * W + col, so the W
// lanes of a launch write each step as one coalesced row.  One lane owns one
// walk: the step loop is a chain of dependent loads (row bounds, then the
// neighbour), and thousands of walks in flight per CU hide that latency.
#include "common.h"
#include "scan.h"

namespace felog {

// --------------------------------------------------------------------------
// Graph validation: one thread per CSR entry.  Records the smallest offending
// row and the kind of fault as (row << 3 | code) with an atomic minimum.
// --------------------------------------------------------------------------
__device__ __forceinline__ int64_t row_of_entry(const int64_t* indptr, int32_t n, int64_t e)
{
    int32_t lo = 0, hi = n - 1;   // last row r with indptr[r] <= e
    while (lo < hi) {
        int32_t mid = lo + (hi - lo + 1) / 2;
        if (indptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t find_in_row(const int64_t* indptr, const int32_t* indices,
                                               int32_t row, int32_t x)
{
    int64_t lo = indptr[row], hi = indptr[row + 1];
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (indices[mid] < x) lo = mid + 1; else hi = mid;
    }
    return (lo < indptr[row + 1] && indices[lo] == x) ? lo : -1;
}

__global__ void validate_graph_kernel(const int64_t* indptr, const int32_t* indices,
                                      const float* weights, int32_t n, int64_t nnz,
                                      unsigned long long* bad)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int32_t u = (int32_t)row_of_entry(indptr, n, e);
    int32_t v = indices[e];
    int code = 0;
    if (v < 0 || v >= n) code = 1;
    else if (v == u) code = 2;
    else if (e > indptr[u] && indices[e - 1] >= v) code = 3;
    else {
        int64_t r = find_in_row(indptr, indices, v, u);
        if (r < 0) code = 4;
        else if (weights) {
            float w = weights[e];
            if (!(w > 0.0f) || !isfinite(w)) code = 5;
            else if (weights[r] != w) code = 6;
        }
    }
    if (code) atomicMin(bad, ((unsigned long long)u << 3) | (unsigned long long)code);
}

void launch_validate_graph(Graph& g, unsigned long long* d_bad)
{
    Ctx& c = *g.ctx;
    FELOG_HIP(hipMemsetAsync(d_bad, 0xFF, sizeof(unsigned long long), c.stream));
    if (g.nnz == 0) return;
    int64_t blocks = (g.nnz + 255) / 256;
    hipLaunchKernelGGL(validate_graph_kernel, dim3(blocks), dim3(256), 0, c.stream,
                       g.indptr.as<int64_t>(), g.indices.as<int32_t>(),
                       g.weighted ? g.weights.as<float>() : nullptr, g.n, g.nnz, d_bad);
    FELOG_HIP(hipGetLastError());
}

// Largest edge weight of each row (1 for unweighted graphs): the rejection bound.
__global__ void row_wmax_kernel(const int64_t* indptr, const float* weights, int32_t n,
                                float* wmax)
{
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    float m = 0.0f;
    if (weights) {
        for (int64_t e = indptr[v]; e < indptr[v + 1]; ++e) m = fmaxf(m, weights[e]);
    } else {
        m = indptr[v + 1] > indptr[v] ? 1.0f : 0.0f;
    }
    wmax[v] = m;
}

void launch_row_wmax(Graph& g)
{
    Ctx& c = *g.ctx;
    g.wmax.alloc(&c, sizeof(float) * g.n);
    hipLaunchKernelGGL(row_wmax_kernel, dim3((g.n + 255) / 256), dim3(256), 0, c.stream,
                       g.indptr.as<int64_t>(), g.weighted ? g.weights.as<float>() : nullptr, g.n,
                       g.wmax.as<float>());
    FELOG_HIP(hipGetLastError());
}

// (index, weight) records of a weighted graph's entries.  A node2vec attempt
// reads the proposal's index and weight; from two arrays that is two random
// cache lines, from one record one.  The walk kernel is bound by such random
// line fetches: with p = 0.5, q = 2 and weights in (0, 1] most proposals are
// rejected, so a step takes several attempts.
__global__ void edge_records_kernel(const int32_t* __restrict__ indices,
                                    const float* __restrict__ weights, int64_t nnz,
                                    int2* __restrict__ edges)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) edges[e] = make_int2(indices[e], __float_as_int(weights[e]));
}

void build_edge_records(Graph& g)
{
    Ctx& c = *g.ctx;
    if (!g.weighted) return;
    g.edges.alloc(&c, sizeof(int2) * std::max<int64_t>(g.nnz, 1));
    if (g.nnz)
        hipLaunchKernelGGL(edge_records_kernel, dim3((g.nnz + 255) / 256), dim3(256), 0,
                           c.stream, g.indices.as<int32_t>(), g.weights.as<float>(), g.nnz,
                           g.edges.as<int2>());
    FELOG_HIP(hipGetLastError());
    c.sync();
    g.weights.release();
}

// --------------------------------------------------------------------------
// Uniform walks.  Transition t of walk `wid` moves from v to its neighbour
// number floor(x0 * deg(v) / 2^32), x0 = word 0 of Philox(wid, t, WALK).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void walk_uniform_kernel(
    const int64_t* __restrict__ indptr, const int32_t* __restrict__ indices,
    const int32_t* __restrict__ starts, int64_t n_starts, int64_t W, int64_t col0,
    int64_t col_end, int32_t L, uint64_t seed, int64_t id_base, int32_t* __restrict__ walks)
{
    int64_t col = col0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= col_end) return;
    int64_t si = col % n_starts;
    int32_t v = starts ? starts[si] : (int32_t)si;
    int64_t wid = id_base + col;
    walks[col] = v;
    int32_t t = 0;
    for (; t + 1 < L; ++t) {
        int64_t lo = indptr[v];
        int64_t deg = indptr[v + 1] - lo;
        if (deg == 0) break;
        Rand4 r = philox4x32((uint32_t)wid, (uint32_t)(wid >> 32), (uint32_t)t, kTagWalk, seed);
        v = indices[lo + scale32(r.v[0], (uint32_t)deg)];
        walks[(int64_t)(t + 1) * W + col] = v;
    }
    for (int32_t s = t + 1; s < L; ++s) walks[(int64_t)s * W + col] = -1;
}

// --------------------------------------------------------------------------
// node2vec walks by rejection.  From v (previous node `prev`), attempt a of
// transition t uses Philox(wid, t, N2V | a): propose the neighbour
// floor(x0 * deg / 2^32), draw u = (x1 >> 8) * 2^-24, and accept when
//   u * (wmax(v) * alpha_max) < w(v, x) * alpha(prev, x)
// in FP32, alpha = 1/p (x == prev), 1 (x adjacent to prev), 1/q (otherwise).
// The first transition uses alpha = 1 and the bound wmax(v).  The adjacency
// test is a binary search in the shorter of the sorted rows of prev and x
// (the graph is symmetric), and it is skipped when the proposal is decided
// by the extreme alpha values alone (same result).
//
// The transition takes the first accepted attempt in attempt order, or after
// max_attempts rejections the last proposal.  Attempts are evaluated S at a
// time: their record reads are issued together, the searches of the
// undecided ones run in lockstep, and the first accepted attempt of the group
// (in order) is taken.  Every attempt keeps its own counter, so the walk is
// the one that evaluating attempt by attempt gives; with most proposals
// rejected (p = 0.5, q = 2, weights in (0, 1]), pairs of attempts save round
// trips to memory (S = 2 keeps 8 waves per SIMD; S = 4 drops to 5 and was
// slower).
// --------------------------------------------------------------------------
constexpr int kN2vAttempts = 2;   // attempts evaluated per round trip

template <int S>
__global__ __launch_bounds__(256) void walk_node2vec_kernel(
    const int64_t* __restrict__ indptr, const int32_t* __restrict__ indices,
    const int2* __restrict__ edges, const float* __restrict__ wmax,
    const int32_t* __restrict__ starts, int64_t n_starts, int64_t W, int64_t col0,
    int64_t col_end, int32_t L, float inv_p, float inv_q, float amax, uint32_t max_attempts,
    uint64_t seed, int64_t id_base, int32_t* __restrict__ walks,
    unsigned long long* __restrict__ capped)
{
    int64_t col = col0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= col_end) return;
    int64_t si = col % n_starts;
    int32_t v = starts ? starts[si] : (int32_t)si;
    int32_t prev = -1;
    int64_t wid = id_base + col;
    walks[col] = v;
    uint32_t my_capped = 0;
    const float a_hi = fmaxf(1.0f, inv_q), a_lo = fminf(1.0f, inv_q);
    int32_t t = 0;
    for (; t + 1 < L; ++t) {
        const int64_t lo = indptr[v];
        const int64_t deg = indptr[v + 1] - lo;
        if (deg == 0) break;
        const float bound = t == 0 ? wmax[v] : __fmul_rn(wmax[v], amax);
        int64_t plo = 0, phi = 0;
        if (t > 0) {
            plo = indptr[prev];
            phi = indptr[prev + 1];
        }
        int32_t x = -1;
        bool done = false;
        for (uint32_t a0 = 0; a0 < max_attempts && !done; a0 += S) {
            int32_t xs[S];     // proposals
            float ws[S], lhs[S];
            int st[S];         // 0 rejected, 1 accepted, 2 decided by adjacency to prev
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const Rand4 r = philox4x32((uint32_t)wid, (uint32_t)(wid >> 32), (uint32_t)t,
                                           kTagN2V | (a0 + (uint32_t)k), seed);
                const int64_t e = lo + scale32(r.v[0], (uint32_t)deg);
                if (edges) {
                    const int2 rec = edges[e];
                    xs[k] = rec.x;
                    ws[k] = __int_as_float(rec.y);
                } else {
                    xs[k] = indices[e];
                    ws[k] = 1.0f;
                }
                lhs[k] = __fmul_rn((float)(r.v[1] >> 8) * (1.0f / 16777216.0f), bound);
            }
            bool any_adj = false;
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (t == 0) st[k] = lhs[k] < ws[k] ? 1 : 0;
                else if (xs[k] == prev) st[k] = lhs[k] < __fmul_rn(ws[k], inv_p) ? 1 : 0;
                else if (!(lhs[k] < __fmul_rn(ws[k], a_hi))) st[k] = 0;
                else if (lhs[k] < __fmul_rn(ws[k], a_lo)) st[k] = 1;
                else st[k] = 2;
                any_adj = any_adj || st[k] == 2;
            }
            if (any_adj) {
                // lower-bound searches of the undecided proposals, each in the
                // shorter of the rows of prev and x for the other node, in
                // lockstep: every round reads one index per search (inactive
                // searches re-read prev's first entry)
                int64_t l[S], h[S], en[S];
                int32_t tg[S];
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    l[k] = plo;
                    h[k] = plo;
                    tg[k] = 0;
                    if (st[k] == 2) {
                        const int64_t xlo = indptr[xs[k]], xhi = indptr[xs[k] + 1];
                        const bool in_x = xhi - xlo < phi - plo;
                        l[k] = in_x ? xlo : plo;
                        h[k] = in_x ? xhi : phi;
                        tg[k] = in_x ? prev : xs[k];
                    }
                    en[k] = h[k];
                }
                for (;;) {
                    bool active = false;
                    int32_t val[S];
                    int64_t mid[S];
#pragma unroll
                    for (int k = 0; k < S; ++k) {
                        mid[k] = l[k] + ((h[k] - l[k]) >> 1);
                        val[k] = indices[l[k] < h[k] ? mid[k] : plo];
                    }
#pragma unroll
                    for (int k = 0; k < S; ++k) {
                        if (l[k] < h[k]) {
                            active = true;
                            if (val[k] < tg[k]) l[k] = mid[k] + 1;
                            else h[k] = mid[k];
                        }
                    }
                    if (!active) break;
                }
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    if (st[k] == 2) {
                        const bool adj = l[k] < en[k] && indices[l[k] < en[k] ? l[k] : plo] == tg[k];
                        st[k] = lhs[k] < __fmul_rn(ws[k], adj ? 1.0f : inv_q) ? 1 : 0;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (!done && a0 + (uint32_t)k < max_attempts) {
                    x = xs[k];
                    done = st[k] == 1;
                }
            }
        }
        if (!done) ++my_capped;
        prev = v;
        v = x;
        walks[(int64_t)(t + 1) * W + col] = v;
    }
    for (int32_t s = t + 1; s < L; ++s) walks[(int64_t)s * W + col] = -1;
    if (my_capped) atomicAdd(capped, (unsigned long long)my_capped);
}

void launch_walk_columns(Walks& w, const felog_walk_params& p, const Active* starts,
                         int64_t n_starts, int64_t col0, int64_t ncols, hipStream_t s,
                         unsigned long long* d_capped)
{
    Graph& g = *w.g;
    FELOG_REQUIRE(col0 >= 0 && ncols >= 0 && col0 + ncols <= w.W, "walk columns out of range");
    if (ncols == 0) return;
    const int32_t* st = starts ? starts->nodes.as<int32_t>() : nullptr;
    const int64_t blocks = (ncols + 255) / 256;
    if (p.kind == FELOG_WALK_UNIFORM) {
        hipLaunchKernelGGL(walk_uniform_kernel, dim3(blocks), dim3(256), 0, s,
                           g.indptr.as<int64_t>(), g.indices.as<int32_t>(), st, n_starts, w.W,
                           col0, col0 + ncols, w.L, p.seed, w.id_base, w.data.as<int32_t>());
    } else {
        FELOG_REQUIRE(d_capped, "node2vec walks need a device counter for capped proposals");
        float inv_p = 1.0f / p.p, inv_q = 1.0f / p.q;
        float amax = fmaxf(1.0f, fmaxf(inv_p, inv_q));
        hipLaunchKernelGGL(walk_node2vec_kernel<kN2vAttempts>, dim3(blocks), dim3(256), 0, s,
                           g.indptr.as<int64_t>(), g.indices.as<int32_t>(),
                           g.weighted ? g.edges.as<int2>() : nullptr, g.wmax.as<float>(), st,
                           n_starts, w.W, col0, col0 + ncols, w.L, inv_p, inv_q, amax, 1u << 16,
                           p.seed, w.id_base, w.data.as<int32_t>(), d_capped);
    }
    FELOG_HIP(hipGetLastError());
}

void launch_walks(Walks& w, const felog_walk_params& p, const Active* starts, int64_t n_starts)
{
    Ctx& c = *w.g->ctx;
    w.have_valid = false;
    w.capped = 0;
    if (p.kind == FELOG_WALK_UNIFORM) {
        launch_walk_columns(w, p, starts, n_starts, 0, w.W, c.stream, nullptr);
        return;
    }
    DevBuf cap;
    cap.alloc(&c, sizeof(unsigned long long));
    FELOG_HIP(hipMemsetAsync(cap.ptr, 0, sizeof(unsigned long long), c.stream));
    launch_walk_columns(w, p, starts, n_starts, 0, w.W, c.stream, cap.as<unsigned long long>());
    unsigned long long h = 0;
    FELOG_HIP(hipMemcpyAsync(&h, cap.ptr, sizeof h, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    w.capped = (int64_t)h;
}

// --------------------------------------------------------------------------
// Columns whose walk yields pairs (two or more nodes), and their count per
// chunk of `chunk` consecutive walks.
// --------------------------------------------------------------------------
struct LongWalk {
    const int32_t* second_step;   // walk[1][*]
    __device__ bool operator()(int64_t col) const { return second_step[col] >= 0; }
};
struct ColumnId {
    __device__ int32_t operator()(int64_t col) const { return (int32_t)col; }
};

// Walks per chunk that yield pairs: valid_cols is sorted, so the count of chunk
// c is the number of entries in [c * chunk, (c + 1) * chunk), by binary search.
__global__ void chunk_count_kernel(const int32_t* valid_cols, int64_t n_valid, int64_t n_chunks,
                                   int64_t chunk, unsigned long long* counts)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    auto lower = [&](int64_t x) {
        int64_t lo = 0, hi = n_valid;
        while (lo < hi) {
            int64_t mid = lo + ((hi - lo) >> 1);
            if (valid_cols[mid] < x) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    counts[c] = (unsigned long long)(lower((c + 1) * chunk) - lower(c * chunk));
}

// valid_cols of the columns with pred(col), and their counts per chunk
template <class Pred>
static void set_valid_columns(Walks& w, int64_t chunk, Pred pred)
{
    Ctx& c = *w.g->ctx;
    int64_t n_chunks = (w.W + chunk - 1) / chunk;
    w.chunk_valid.assign(n_chunks, 0);
    if (w.L < 2 || w.W == 0) {
        w.n_valid = 0;
        w.valid_cols.alloc(&c, sizeof(int32_t));
    } else {
        w.n_valid = compact(c, pred, ColumnId{}, w.W, w.valid_cols);
        DevBuf cnt;
        cnt.alloc(&c, sizeof(unsigned long long) * n_chunks);
        hipLaunchKernelGGL(chunk_count_kernel, dim3((n_chunks + 255) / 256), dim3(256), 0,
                           c.stream, w.valid_cols.as<int32_t>(), w.n_valid, n_chunks, chunk,
                           cnt.as<unsigned long long>());
        FELOG_HIP(hipGetLastError());
        std::vector<unsigned long long> h(n_chunks);
        FELOG_HIP(hipMemcpyAsync(h.data(), cnt.ptr, sizeof(unsigned long long) * n_chunks,
                                 hipMemcpyDeviceToHost, c.stream));
        c.sync();
        for (int64_t i = 0; i < n_chunks; ++i) w.chunk_valid[i] = (int64_t)h[i];
    }
    w.have_valid = true;
    w.chunk_for_valid = chunk;
}

void launch_valid_columns(Walks& w, int64_t chunk)
{
    if (w.have_valid && w.chunk_for_valid == chunk) return;
    set_valid_columns(w, chunk, LongWalk{w.data.as<int32_t>() + w.W});
}

// A walk has a second node exactly when its start node has a neighbour: both
// samplers stop only at a node without neighbours, and node2vec takes its last
// proposal when every attempt is rejected.  So the columns that yield pairs are
// known from the start list alone, before any walk is written.
struct StartHasNeighbour {
    const int64_t* indptr;
    const int32_t* starts;    // null: start of column col is col mod n_starts
    int64_t n_starts;
    __device__ bool operator()(int64_t col) const
    {
        const int64_t si = col % n_starts;
        const int32_t v = starts ? starts[si] : (int32_t)si;
        return indptr[v + 1] > indptr[v];
    }
};

void plan_valid_columns(Walks& w, const Active* starts, int64_t n_starts, int64_t chunk)
{
    const Graph& g = *w.g;
    set_valid_columns(w, chunk, StartHasNeighbour{g.indptr.as<int64_t>(),
                                                  starts ? starts->nodes.as<int32_t>() : nullptr,
                                                  n_starts});
}

}  // namespace felog
