// C ABI of the FeLoG hot path (include/felog.h): argument checks, handle
// lifetimes, host<->device copies and Algorithm 1's round loop.  Every step
// of the method runs in the kernels of the .hip files.
#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>

#include "common.h"

struct felog_ctx : felog::Ctx {};
struct felog_graph : felog::Graph {};
struct felog_walks : felog::Walks {};
struct felog_packed : felog::Packed {};
struct felog_active : felog::Active {};
struct felog_model : felog::Model {};

namespace felog {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

void fail(felog_status code, const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    throw Error{code};
}

DevBuf& DevBuf::operator=(DevBuf&& o) noexcept
{
    if (this != &o) {
        release();
        ctx = o.ctx;
        ptr = o.ptr;
        bytes = o.bytes;
        o.ctx = nullptr;
        o.ptr = nullptr;
        o.bytes = 0;
    }
    return *this;
}

void DevBuf::alloc(Ctx* c, size_t nbytes)
{
    release();
    if (nbytes == 0) nbytes = 16;
    if (c->budget && c->in_use + nbytes > c->budget)
        fail(FELOG_ENOMEM, "HBM budget exceeded: %llu bytes held, %llu requested, budget %llu",
             (unsigned long long)c->in_use, (unsigned long long)nbytes,
             (unsigned long long)c->budget);
    c->make_current();
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess)
        fail(FELOG_ENOMEM, "hipMalloc(%llu) failed: %s", (unsigned long long)nbytes,
             hipGetErrorString(e));
    ctx = c;
    ptr = p;
    bytes = nbytes;
    c->in_use += nbytes;
    c->peak = std::max(c->peak, c->in_use);
}

void DevBuf::release()
{
    if (ptr) {
        ctx->make_current();
        (void)hipFree(ptr);
        ctx->in_use -= bytes;
    }
    ptr = nullptr;
    bytes = 0;
    ctx = nullptr;
}

void Ctx::make_current() const { (void)hipSetDevice(device); }

void Ctx::sync() const { FELOG_HIP(hipStreamSynchronize(stream)); }

void Ctx::ensure_aux()
{
    if (aux) return;
    make_current();
    if (single_stream)
        aux = stream;
    else
        FELOG_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
    for (hipEvent_t& e : pipe_ev) FELOG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

void Ctx::release_aux()
{
    if (!aux) return;
    make_current();
    (void)hipStreamSynchronize(aux);
    for (hipEvent_t& e : pipe_ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (aux != stream) (void)hipStreamDestroy(aux);
    aux = nullptr;
}

}  // namespace felog

using namespace felog;

// Run `body`, turning thrown errors into status codes.
template <class F>
static felog_status guarded(F&& body)
{
    clear_error();
    try {
        body();
        return FELOG_OK;
    } catch (const Error& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return FELOG_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return FELOG_EDEVICE;
    }
}

#define NEED(p) FELOG_REQUIRE((p) != nullptr, "%s must not be NULL", #p)

// A model on g with freshly initialised tables (and the degree noise table
// when asked for); throws on a bad parameter.
static std::unique_ptr<felog_model> new_model(felog_graph* g, const felog_model_params* p)
{
    FELOG_REQUIRE(p->dim == 64 || p->dim == 128 || p->dim == 256,
                  "dim must be 64, 128 or 256 (got %d)", p->dim);
    FELOG_REQUIRE(p->neg_dist == FELOG_NEG_DEGREE || p->neg_dist == FELOG_NEG_UNIGRAM,
                  "unknown noise distribution %d", p->neg_dist);
    FELOG_REQUIRE(p->precision == FELOG_PREC_FP32 || p->precision == FELOG_PREC_BF16,
                  "unknown precision %d", p->precision);
    Ctx* c = g->ctx;
    auto m = std::make_unique<felog_model>();
    m->ctx = c;
    m->g = g;
    m->dim = p->dim;
    m->neg_dist = p->neg_dist;
    m->precision = p->precision;
    size_t tb = sizeof(float) * (size_t)g->n * p->dim;
    m->tin.alloc(c, tb);
    m->tout.alloc(c, tb);
    model_alloc_update_state(*m);
    if (p->precision == FELOG_PREC_BF16) {
        m->bin.alloc(c, sizeof(uint16_t) * (size_t)g->n * p->dim);
        m->bout.alloc(c, sizeof(uint16_t) * (size_t)g->n * p->dim);
    }
    launch_init_tables(*m, p->seed);
    if (p->neg_dist == FELOG_NEG_DEGREE) {
        DevBuf counts;
        counts.alloc(c, sizeof(uint32_t) * g->n);
        launch_degree_counts(*g, counts.as<uint32_t>());
        build_noise_from_counts(*m, counts.as<uint32_t>());
        c->sync();
    }
    c->sync();
    return m;
}

extern "C" {

const char* felog_last_error(void) { return g_last_error.c_str(); }

// ----------------------------------------------------------------- context
felog_status felog_ctx_create(int device, void* hip_stream, uint64_t hbm_budget_bytes,
                              felog_ctx** out)
{
    return guarded([&] {
        NEED(out);
        *out = nullptr;
        int n = 0;
        FELOG_HIP(hipGetDeviceCount(&n));
        FELOG_REQUIRE(device >= 0 && device < n, "device %d out of range (%d devices)", device, n);
        FELOG_HIP(hipSetDevice(device));
        hipDeviceProp_t prop;
        FELOG_HIP(hipGetDeviceProperties(&prop, device));
        auto c = std::make_unique<felog_ctx>();
        c->device = device;
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->budget = hbm_budget_bytes;
        c->num_cus = prop.multiProcessorCount;
        noalloc_scratch_init(device);
        FELOG_HIP(hipEventCreate(&c->ev0));
        FELOG_HIP(hipEventCreate(&c->ev1));
        *out = c.release();
    });
}

void felog_ctx_destroy(felog_ctx* ctx)
{
    if (!ctx) return;
    ctx->make_current();
    (void)hipStreamSynchronize(ctx->stream);
    ctx->release_aux();
    if (ctx->walk_stream) {
        (void)hipStreamSynchronize(ctx->walk_stream);
        (void)hipStreamDestroy(ctx->walk_stream);
    }
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (hipEvent_t e : ctx->timing_pool) (void)hipEventDestroy(e);
    delete ctx;
}

felog_status felog_ctx_set_timing(felog_ctx* ctx, int32_t every)
{
    return guarded([&] {
        NEED(ctx);
        FELOG_REQUIRE(every >= 0, "every must be >= 0");
        ctx->make_current();
        if (every > 0 && ctx->timing_pool.empty()) {
            ctx->timing_pool.resize(kTimingEvents * 256);
            for (hipEvent_t& e : ctx->timing_pool) FELOG_HIP(hipEventCreate(&e));
        }
        ctx->timing_every = every;
    });
}

felog_status felog_ctx_set_sgns_path(felog_ctx* ctx, int32_t path, int32_t blocks)
{
    return guarded([&] {
        NEED(ctx);
        FELOG_REQUIRE(path == 0 || path == 1, "path must be 0 or 1");
        FELOG_REQUIRE(blocks >= 0 && blocks <= 65536, "blocks out of range");
        ctx->sgns_path = path;
        ctx->sgns_blocks = blocks;
    });
}

felog_status felog_ctx_set_single_stream(felog_ctx* ctx, int32_t on)
{
    return guarded([&] {
        NEED(ctx);
        FELOG_REQUIRE(on == 0 || on == 1, "on must be 0 or 1");
        ctx->release_aux();   // waits for the second stream's work
        ctx->single_stream = on != 0;
    });
}

felog_status felog_ctx_bytes_in_use(const felog_ctx* ctx, uint64_t* bytes)
{
    return guarded([&] {
        NEED(ctx);
        NEED(bytes);
        *bytes = ctx->in_use;
    });
}

// ------------------------------------------------------------------- graph
felog_status felog_graph_load_csr(felog_ctx* ctx, int32_t n_nodes, int64_t nnz,
                                  const int64_t* indptr, const int32_t* indices,
                                  const float* weights, felog_graph** out)
{
    return guarded([&] {
        NEED(ctx);
        NEED(out);
        NEED(indptr);
        *out = nullptr;
        FELOG_REQUIRE(n_nodes >= 1, "n_nodes must be >= 1 (got %d)", n_nodes);
        FELOG_REQUIRE(nnz >= 0, "nnz must be >= 0");
        FELOG_REQUIRE(nnz == 0 || indices, "indices must not be NULL when nnz > 0");
        FELOG_REQUIRE(indptr[0] == 0, "indptr[0] must be 0 (got %lld)", (long long)indptr[0]);
        FELOG_REQUIRE(indptr[n_nodes] == nnz, "indptr[n] = %lld differs from nnz = %lld",
                      (long long)indptr[n_nodes], (long long)nnz);
        int64_t isolated = 0;
        for (int32_t v = 0; v < n_nodes; ++v) {
            FELOG_REQUIRE(indptr[v + 1] >= indptr[v], "indptr decreases at row %d", v);
            isolated += indptr[v + 1] == indptr[v];
        }
        ctx->make_current();
        auto g = std::make_unique<felog_graph>();
        g->ctx = ctx;
        g->n = n_nodes;
        g->nnz = nnz;
        g->weighted = weights != nullptr;
        g->isolated = isolated;
        g->indptr.alloc(ctx, sizeof(int64_t) * (n_nodes + 1));
        g->indices.alloc(ctx, sizeof(int32_t) * std::max<int64_t>(nnz, 1));
        FELOG_HIP(hipMemcpyAsync(g->indptr.ptr, indptr, sizeof(int64_t) * (n_nodes + 1),
                                 hipMemcpyHostToDevice, ctx->stream));
        if (nnz)
            FELOG_HIP(hipMemcpyAsync(g->indices.ptr, indices, sizeof(int32_t) * nnz,
                                     hipMemcpyHostToDevice, ctx->stream));
        if (weights) {
            g->weights.alloc(ctx, sizeof(float) * std::max<int64_t>(nnz, 1));
            if (nnz)
                FELOG_HIP(hipMemcpyAsync(g->weights.ptr, weights, sizeof(float) * nnz,
                                         hipMemcpyHostToDevice, ctx->stream));
        }
        DevBuf bad;
        bad.alloc(ctx, sizeof(unsigned long long));
        launch_validate_graph(*g, bad.as<unsigned long long>());
        unsigned long long h_code = 0;
        FELOG_HIP(hipMemcpyAsync(&h_code, bad.ptr, sizeof h_code, hipMemcpyDeviceToHost,
                                 ctx->stream));
        ctx->sync();
        int32_t h_bad[2] = {INT32_MAX, 0};
        if (h_code != ~0ull) {
            h_bad[0] = (int32_t)(h_code >> 3);
            h_bad[1] = (int32_t)(h_code & 7);
        }
        static const char* what[] = {"", "an index out of [0, n)", "a self loop",
                                     "indices not strictly increasing",
                                     "an edge whose reverse is missing",
                                     "a weight that is not positive and finite",
                                     "a weight that differs from its reverse edge's"};
        if (h_bad[0] != INT32_MAX)
            fail(FELOG_EINVAL, "graph is not a valid symmetric CSR: row %d has %s", h_bad[0],
                 what[h_bad[1] >= 0 && h_bad[1] < 7 ? h_bad[1] : 0]);
        launch_row_wmax(*g);
        build_edge_records(*g);
        ctx->sync();
        *out = g.release();
    });
}

void felog_graph_destroy(felog_graph* g) { delete g; }

felog_status felog_graph_info(const felog_graph* g, int32_t* n_nodes, int64_t* nnz,
                              int32_t* weighted)
{
    return guarded([&] {
        NEED(g);
        if (n_nodes) *n_nodes = g->n;
        if (nnz) *nnz = g->nnz;
        if (weighted) *weighted = g->weighted ? 1 : 0;
    });
}

// ------------------------------------------------------------------ active
felog_status felog_active_from_host(felog_graph* g, const int32_t* nodes, int64_t count,
                                    felog_active** out)
{
    return guarded([&] {
        NEED(g);
        NEED(out);
        *out = nullptr;
        FELOG_REQUIRE(count >= 0 && count <= g->n, "count %lld out of range", (long long)count);
        FELOG_REQUIRE(count == 0 || nodes, "nodes must not be NULL when count > 0");
        for (int64_t i = 0; i < count; ++i) {
            FELOG_REQUIRE(nodes[i] >= 0 && nodes[i] < g->n, "node %d at %lld out of range",
                          nodes[i], (long long)i);
            FELOG_REQUIRE(i == 0 || nodes[i] > nodes[i - 1],
                          "active list must be strictly increasing (position %lld)",
                          (long long)i);
        }
        auto a = std::make_unique<felog_active>();
        a->g = g;
        a->count = count;
        a->nodes.alloc(g->ctx, sizeof(int32_t) * std::max<int64_t>(count, 1));
        if (count)
            FELOG_HIP(hipMemcpyAsync(a->nodes.ptr, nodes, sizeof(int32_t) * count,
                                     hipMemcpyHostToDevice, g->ctx->stream));
        g->ctx->sync();
        *out = a.release();
    });
}

felog_status felog_active_all(felog_graph* g, felog_active** out)
{
    return guarded([&] {
        NEED(g);
        NEED(out);
        *out = nullptr;
        std::vector<int32_t> all(g->n);
        for (int32_t v = 0; v < g->n; ++v) all[v] = v;
        auto a = std::make_unique<felog_active>();
        a->g = g;
        a->count = g->n;
        a->nodes.alloc(g->ctx, sizeof(int32_t) * g->n);
        FELOG_HIP(hipMemcpyAsync(a->nodes.ptr, all.data(), sizeof(int32_t) * g->n,
                                 hipMemcpyHostToDevice, g->ctx->stream));
        g->ctx->sync();
        *out = a.release();
    });
}

felog_status felog_active_count(const felog_active* a, int64_t* count)
{
    return guarded([&] {
        NEED(a);
        NEED(count);
        *count = a->count;
    });
}

felog_status felog_active_read(const felog_active* a, int32_t* nodes, int64_t cap,
                               int64_t* count)
{
    return guarded([&] {
        NEED(a);
        if (count) *count = a->count;
        if (a->count == 0) return;
        NEED(nodes);
        FELOG_REQUIRE(cap >= a->count, "buffer holds %lld nodes, need %lld", (long long)cap,
                      (long long)a->count);
        Ctx* c = a->g->ctx;
        FELOG_HIP(hipMemcpyAsync(nodes, a->nodes.ptr, sizeof(int32_t) * a->count,
                                 hipMemcpyDeviceToHost, c->stream));
        c->sync();
    });
}

void felog_active_destroy(felog_active* a) { delete a; }

// ------------------------------------------------------------------- walks
static void check_walk_params(const Graph* g, const felog_walk_params* p)
{
    NEED(p);
    FELOG_REQUIRE(p->kind == FELOG_WALK_UNIFORM || p->kind == FELOG_WALK_NODE2VEC,
                  "unknown walk kind %d", p->kind);
    FELOG_REQUIRE(p->walks_per_node >= 1, "walks_per_node must be >= 1");
    FELOG_REQUIRE(p->length >= 1 && p->length <= 65536, "length must be in [1, 65536]");
    FELOG_REQUIRE(p->id_base >= 0, "id_base must be >= 0");
    if (p->kind == FELOG_WALK_NODE2VEC)
        FELOG_REQUIRE(p->p > 0 && p->q > 0 && std::isfinite(p->p) && std::isfinite(p->q),
                      "node2vec p and q must be positive and finite");
    (void)g;
}

felog_status felog_walks_generate(felog_graph* g, const felog_walk_params* params,
                                  const felog_active* starts, felog_walks** out)
{
    return guarded([&] {
        NEED(g);
        NEED(out);
        *out = nullptr;
        check_walk_params(g, params);
        FELOG_REQUIRE(!starts || starts->g == g, "active set belongs to another graph");
        int64_t n_starts = starts ? starts->count : g->n;
        auto w = std::make_unique<felog_walks>();
        w->g = g;
        w->L = params->length;
        w->W = n_starts * params->walks_per_node;
        w->id_base = params->id_base;
        w->data.alloc(g->ctx, sizeof(int32_t) * std::max<int64_t>(w->W * w->L, 1));
        if (w->W) launch_walks(*w, *params, starts, n_starts);
        g->ctx->sync();
        *out = w.release();
    });
}

felog_status felog_walks_info(const felog_walks* w, int64_t* n_walks, int32_t* length,
                              int64_t* id_base)
{
    return guarded([&] {
        NEED(w);
        if (n_walks) *n_walks = w->W;
        if (length) *length = w->L;
        if (id_base) *id_base = w->id_base;
    });
}

felog_status felog_walks_read_range(const felog_walks* w, int64_t first, int64_t count,
                                    int32_t* walks, int64_t cap)
{
    return guarded([&] {
        NEED(w);
        FELOG_REQUIRE(first >= 0 && count >= 0 && first + count <= w->W,
                      "walks [%lld, %lld) outside [0, %lld)", (long long)first,
                      (long long)(first + count), (long long)w->W);
        const int64_t total = count * w->L;
        if (total == 0) return;
        NEED(walks);
        FELOG_REQUIRE(cap >= total, "buffer holds %lld ints, need %lld", (long long)cap,
                      (long long)total);
        Ctx* c = w->g->ctx;
        // Device layout is step-major [L][W]: one strided copy of the L rows'
        // column range, then a transpose to walk-major on the host.
        std::vector<int32_t> tmp(total);
        FELOG_HIP(hipMemcpy2DAsync(tmp.data(), sizeof(int32_t) * count,
                                   w->data.as<int32_t>() + first, sizeof(int32_t) * w->W,
                                   sizeof(int32_t) * count, w->L, hipMemcpyDeviceToHost,
                                   c->stream));
        c->sync();
        for (int32_t t = 0; t < w->L; ++t)
            for (int64_t col = 0; col < count; ++col)
                walks[col * w->L + t] = tmp[t * count + col];
    });
}

felog_status felog_walks_read(const felog_walks* w, int32_t* walks, int64_t cap)
{
    if (!w) return felog_walks_read_range(w, 0, 0, walks, cap);
    return felog_walks_read_range(w, 0, w->W, walks, cap);
}

felog_status felog_walks_capped(const felog_walks* w, int64_t* capped)
{
    return guarded([&] {
        NEED(w);
        NEED(capped);
        *capped = w->capped;
    });
}

void felog_walks_destroy(felog_walks* w) { delete w; }

// -------------------------------------------------------------- walk codec
felog_status felog_fabc_profile(const felog_walks* w, int32_t k_max, int32_t* k,
                                int32_t* symbols, uint64_t* counts, int32_t* n_ranked,
                                uint64_t* total)
{
    return guarded([&] {
        NEED(w);
        NEED(k);
        NEED(symbols);
        NEED(counts);
        NEED(n_ranked);
        NEED(total);
        FELOG_REQUIRE(k_max >= 0 && k_max <= kFabcMax, "k_max must be in [0, %d]", kFabcMax);
        fabc_profile(*w, k_max, k, symbols, counts, n_ranked, total);
    });
}

felog_status felog_walks_pack(const felog_walks* w, int32_t k, const int32_t* symbols,
                              felog_packed** out, double* ms)
{
    return guarded([&] {
        NEED(w);
        NEED(out);
        *out = nullptr;
        FELOG_REQUIRE(k >= 0 && k <= kFabcMax, "k must be in [0, %d]", kFabcMax);
        if (k > 0) NEED(symbols);
        for (int b = 0; b < k; ++b) {
            FELOG_REQUIRE(symbols[b] >= -1 && symbols[b] < w->g->n,
                          "symbol %d outside [-1, %d)", symbols[b], w->g->n);
            for (int q = 0; q < b; ++q)
                FELOG_REQUIRE(symbols[q] != symbols[b], "symbol %d repeated", symbols[b]);
        }
        auto p = std::make_unique<felog_packed>();
        fabc_pack(*w, k, symbols, *p, ms);
        *out = p.release();
    });
}

felog_status felog_packed_info(const felog_packed* p, int64_t* bytes, int32_t* k,
                               int64_t* n_walks, int32_t* length, int64_t* residuals)
{
    return guarded([&] {
        NEED(p);
        if (bytes) *bytes = p->bytes;
        if (k) *k = p->k;
        if (n_walks) *n_walks = p->W;
        if (length) *length = p->L;
        if (residuals) *residuals = p->R;
    });
}

felog_status felog_packed_read(const felog_packed* p, void* host, int64_t cap)
{
    return guarded([&] {
        NEED(p);
        NEED(host);
        FELOG_REQUIRE(cap >= p->bytes, "buffer holds %lld bytes, need %lld", (long long)cap,
                      (long long)p->bytes);
        Ctx* c = p->g->ctx;
        c->make_current();
        FELOG_HIP(hipMemcpyAsync(host, p->buf.ptr, (size_t)p->bytes, hipMemcpyDeviceToHost,
                                 c->stream));
        c->sync();
    });
}

felog_status felog_packed_from_host(felog_graph* g, const void* host, int64_t bytes,
                                    felog_packed** out)
{
    return guarded([&] {
        NEED(g);
        NEED(host);
        NEED(out);
        *out = nullptr;
        auto p = std::make_unique<felog_packed>();
        fabc_from_host(*g, host, bytes, *p);
        *out = p.release();
    });
}

felog_status felog_packed_unpack(const felog_packed* p, felog_walks** out, double* ms)
{
    return guarded([&] {
        NEED(p);
        NEED(out);
        *out = nullptr;
        auto w = std::make_unique<felog_walks>();
        fabc_unpack(*p, *w, ms);
        *out = w.release();
    });
}

void felog_packed_destroy(felog_packed* p) { delete p; }

// ------------------------------------------------------------------- model
felog_status felog_model_create(felog_graph* g, const felog_model_params* p, felog_model** out)
{
    return guarded([&] {
        NEED(g);
        NEED(p);
        NEED(out);
        *out = nullptr;
        *out = new_model(g, p).release();
    });
}

void felog_model_destroy(felog_model* m) { delete m; }

felog_status felog_model_reset(felog_model* m, uint64_t seed)
{
    return guarded([&] {
        NEED(m);
        launch_init_tables(*m, seed);
        if (m->neg_dist == FELOG_NEG_UNIGRAM) m->have_noise = false;
        m->ctx->sync();
    });
}

felog_status felog_model_info(const felog_model* m, int32_t* n, int32_t* dim, int32_t* neg_dist,
                              int32_t* precision)
{
    return guarded([&] {
        NEED(m);
        if (n) *n = m->g->n;
        if (dim) *dim = m->dim;
        if (neg_dist) *neg_dist = m->neg_dist;
        if (precision) *precision = m->precision;
    });
}

// ------------------------------------------------------------ checkpoints
constexpr uint32_t kCheckpointMagic = 0x4D4C6546u;   // "FeLM"
constexpr uint32_t kCheckpointVersion = 1;
struct CheckpointHeader {
    uint32_t magic, version;
    int32_t n, dim, neg_dist, precision;
    uint32_t round, flags;
    int64_t walk_id_base, n_active;
    uint64_t nnz, zero;
};
static_assert(sizeof(CheckpointHeader) == 64, "checkpoint header is 64 bytes");

struct File {
    std::FILE* f = nullptr;
    const char* path;
    File(const char* p, const char* mode) : f(std::fopen(p, mode)), path(p)
    {
        if (!f) fail(FELOG_EIO, "cannot open %s: %s", p, std::strerror(errno));
    }
    ~File()
    {
        if (f) std::fclose(f);
    }
    void write(const void* data, size_t bytes)
    {
        if (bytes && std::fwrite(data, 1, bytes, f) != bytes)
            fail(FELOG_EIO, "writing %s failed", path);
    }
    void read(void* data, size_t bytes)
    {
        if (bytes && std::fread(data, 1, bytes, f) != bytes)
            fail(FELOG_EIO, "%s ends early (truncated checkpoint)", path);
    }
    void close()
    {
        const int e = std::fclose(f);
        f = nullptr;
        if (e != 0) fail(FELOG_EIO, "closing %s failed", path);
    }
};

felog_status felog_model_save(const felog_model* m, const felog_active* active,
                              const felog_checkpoint_meta* meta, const char* path)
{
    return guarded([&] {
        NEED(m);
        NEED(path);
        FELOG_REQUIRE(!active || active->g == m->g, "active set belongs to another graph");
        Ctx* c = m->ctx;
        const int32_t n = m->g->n;
        const size_t cnt = (size_t)n * m->dim;
        CheckpointHeader h{};
        h.magic = kCheckpointMagic;
        h.version = kCheckpointVersion;
        h.n = n;
        h.dim = m->dim;
        h.neg_dist = m->neg_dist;
        h.precision = m->precision;
        h.round = meta ? meta->round : 0u;
        h.flags = (m->have_noise ? 1u : 0u) | (active ? 2u : 0u);
        h.walk_id_base = meta ? meta->walk_id_base : 0;
        h.n_active = active ? active->count : 0;
        h.nnz = (uint64_t)m->g->nnz;
        std::vector<float> tab(std::max<size_t>(cnt, 1));
        File f(path, "wb");
        f.write(&h, sizeof h);
        for (const DevBuf* t : {&m->tin, &m->tout}) {
            FELOG_HIP(hipMemcpyAsync(tab.data(), t->ptr, sizeof(float) * cnt,
                                     hipMemcpyDeviceToHost, c->stream));
            c->sync();
            f.write(tab.data(), sizeof(float) * cnt);
        }
        if (m->have_noise) {
            std::vector<uint64_t> cdf((size_t)n + 1);
            FELOG_HIP(hipMemcpyAsync(cdf.data(), m->cdf.ptr, sizeof(uint64_t) * (n + 1),
                                     hipMemcpyDeviceToHost, c->stream));
            c->sync();
            f.write(cdf.data(), sizeof(uint64_t) * (n + 1));
        }
        if (active && active->count) {
            std::vector<int32_t> nodes(active->count);
            FELOG_HIP(hipMemcpyAsync(nodes.data(), active->nodes.ptr,
                                     sizeof(int32_t) * active->count, hipMemcpyDeviceToHost,
                                     c->stream));
            c->sync();
            f.write(nodes.data(), sizeof(int32_t) * active->count);
        }
        f.close();
    });
}

felog_status felog_model_load(felog_graph* g, const char* path, felog_model** out,
                              felog_active** active, felog_checkpoint_meta* meta)
{
    return guarded([&] {
        NEED(g);
        NEED(path);
        NEED(out);
        *out = nullptr;
        if (active) *active = nullptr;
        File f(path, "rb");
        CheckpointHeader h{};
        f.read(&h, sizeof h);
        FELOG_REQUIRE(h.magic == kCheckpointMagic, "%s is not a model checkpoint", path);
        FELOG_REQUIRE(h.version == kCheckpointVersion, "checkpoint version %u is not supported",
                      h.version);
        FELOG_REQUIRE(h.n == g->n && h.nnz == (uint64_t)g->nnz,
                      "the checkpoint is of a graph with %d nodes and %llu entries, not %d and "
                      "%lld", h.n, (unsigned long long)h.nnz, g->n, (long long)g->nnz);
        FELOG_REQUIRE((h.flags & ~3u) == 0 && h.zero == 0, "unknown checkpoint flags");
        FELOG_REQUIRE(h.n_active >= 0 && h.n_active <= h.n && ((h.flags & 2u) || !h.n_active),
                      "bad active count %lld", (long long)h.n_active);
        const size_t cnt = (size_t)h.n * (size_t)std::max(h.dim, 0);
        const uint64_t expect = sizeof h + 2 * sizeof(float) * cnt +
                                ((h.flags & 1u) ? sizeof(uint64_t) * ((uint64_t)h.n + 1) : 0) +
                                sizeof(int32_t) * (uint64_t)h.n_active;
        FELOG_REQUIRE(std::fseek(f.f, 0, SEEK_END) == 0, "cannot seek in %s", path);
        const long size = std::ftell(f.f);
        FELOG_REQUIRE(size >= 0 && (uint64_t)size == expect,
                      "%s holds %ld bytes; its header describes %llu", path, size,
                      (unsigned long long)expect);
        FELOG_REQUIRE(std::fseek(f.f, (long)sizeof h, SEEK_SET) == 0, "cannot seek in %s", path);
        felog_model_params prm{h.dim, h.neg_dist, 0, h.precision};
        std::unique_ptr<felog_model> m = new_model(g, &prm);   // checks d, noise, precision
        Ctx* c = g->ctx;
        std::vector<float> tab(std::max<size_t>(cnt, 1));
        for (DevBuf* t : {&m->tin, &m->tout}) {
            f.read(tab.data(), sizeof(float) * cnt);
            FELOG_HIP(hipMemcpyAsync(t->ptr, tab.data(), sizeof(float) * cnt,
                                     hipMemcpyHostToDevice, c->stream));
            c->sync();
        }
        if (h.flags & 1u) {
            std::vector<uint64_t> cdf((size_t)h.n + 1);
            f.read(cdf.data(), sizeof(uint64_t) * cdf.size());
            set_noise_cdf(*m, cdf.data());
        } else {
            m->have_noise = false;
        }
        std::unique_ptr<felog_active> a;
        if (h.flags & 2u) {
            std::vector<int32_t> nodes(std::max<int64_t>(h.n_active, 1));
            f.read(nodes.data(), sizeof(int32_t) * h.n_active);
            for (int64_t i = 0; i < h.n_active; ++i)
                FELOG_REQUIRE(nodes[i] >= 0 && nodes[i] < g->n && (i == 0 || nodes[i] > nodes[i - 1]),
                              "the saved active list is not sorted and in range (position %lld)",
                              (long long)i);
            a = std::make_unique<felog_active>();
            a->g = g;
            a->count = h.n_active;
            a->nodes.alloc(c, sizeof(int32_t) * std::max<int64_t>(h.n_active, 1));
            if (h.n_active)
                FELOG_HIP(hipMemcpyAsync(a->nodes.ptr, nodes.data(), sizeof(int32_t) * h.n_active,
                                         hipMemcpyHostToDevice, c->stream));
            c->sync();
        }
        if (meta) {
            meta->round = h.round;
            meta->walk_id_base = h.walk_id_base;
        }
        if (active) *active = a.release();
        *out = m.release();
    });
}

felog_status felog_model_set_unigram(felog_model* m, const felog_walks* corpus)
{
    return guarded([&] {
        NEED(m);
        NEED(corpus);
        FELOG_REQUIRE(corpus->g == m->g, "corpus belongs to another graph");
        Ctx* c = m->ctx;
        DevBuf counts;
        counts.alloc(c, sizeof(uint32_t) * m->g->n);
        launch_corpus_counts(*corpus, counts.as<uint32_t>());
        build_noise_from_counts(*m, counts.as<uint32_t>());
        c->sync();
    });
}

felog_status felog_model_read_cdf(const felog_model* m, uint64_t* cdf, int64_t cap)
{
    return guarded([&] {
        NEED(m);
        NEED(cdf);
        FELOG_REQUIRE(m->have_noise, "the noise distribution is not set yet");
        FELOG_REQUIRE(cap >= (int64_t)m->g->n + 1, "buffer holds %lld values, need %d",
                      (long long)cap, m->g->n + 1);
        FELOG_HIP(hipMemcpyAsync(cdf, m->cdf.ptr, sizeof(uint64_t) * (m->g->n + 1),
                                 hipMemcpyDeviceToHost, m->ctx->stream));
        m->ctx->sync();
    });
}

static const DevBuf& table_of(const felog_model* m, int32_t which)
{
    FELOG_REQUIRE(which == FELOG_TABLE_IN || which == FELOG_TABLE_OUT, "unknown table %d", which);
    return which == FELOG_TABLE_IN ? m->tin : m->tout;
}

felog_status felog_embeddings_read(const felog_model* m, int32_t which, float* host, int64_t cap)
{
    return guarded([&] {
        NEED(m);
        NEED(host);
        const DevBuf& t = table_of(m, which);
        int64_t count = (int64_t)m->g->n * m->dim;
        FELOG_REQUIRE(cap >= count, "buffer holds %lld floats, need %lld", (long long)cap,
                      (long long)count);
        FELOG_HIP(hipMemcpyAsync(host, t.ptr, sizeof(float) * count, hipMemcpyDeviceToHost,
                                 m->ctx->stream));
        m->ctx->sync();
    });
}

felog_status felog_embeddings_read_dev(const felog_model* m, int32_t which, void* dev,
                                       int64_t cap)
{
    return guarded([&] {
        NEED(m);
        NEED(dev);
        const DevBuf& t = table_of(m, which);
        int64_t count = (int64_t)m->g->n * m->dim;
        FELOG_REQUIRE(cap >= count, "buffer holds %lld floats, need %lld", (long long)cap,
                      (long long)count);
        FELOG_HIP(hipMemcpyAsync(dev, t.ptr, sizeof(float) * count, hipMemcpyDeviceToDevice,
                                 m->ctx->stream));
        m->ctx->sync();
    });
}

felog_status felog_embeddings_write(felog_model* m, int32_t which, const float* host,
                                    int64_t count)
{
    return guarded([&] {
        NEED(m);
        NEED(host);
        const DevBuf& t = table_of(m, which);
        FELOG_REQUIRE(count == (int64_t)m->g->n * m->dim, "count must be n * d = %lld",
                      (long long)m->g->n * m->dim);
        FELOG_HIP(hipMemcpyAsync(t.ptr, host, sizeof(float) * count, hipMemcpyHostToDevice,
                                 m->ctx->stream));
        m->ctx->sync();
    });
}

felog_status felog_embeddings_read_bf16(const felog_model* m, int32_t which, uint16_t* host,
                                        int64_t cap)
{
    return guarded([&] {
        NEED(m);
        NEED(host);
        FELOG_REQUIRE(m->precision == FELOG_PREC_BF16, "the model has no BF16 tables");
        FELOG_REQUIRE(which == FELOG_TABLE_IN || which == FELOG_TABLE_OUT, "unknown table %d",
                      which);
        int64_t count = (int64_t)m->g->n * m->dim;
        FELOG_REQUIRE(cap >= count, "buffer holds %lld values, need %lld", (long long)cap,
                      (long long)count);
        bf16_refresh_all(*const_cast<felog_model*>(m));   // round the masters as they stand
        FELOG_HIP(hipMemcpyAsync(host, (which == FELOG_TABLE_IN ? m->bin : m->bout).ptr,
                                 sizeof(uint16_t) * count, hipMemcpyDeviceToHost, m->ctx->stream));
        m->ctx->sync();
    });
}

// ------------------------------------------------------------------- train
static void check_train_params(const felog_model* m, const felog_walks* w,
                               const felog_train_params* p)
{
    NEED(m);
    NEED(w);
    NEED(p);
    FELOG_REQUIRE(w->g == m->g, "corpus belongs to another graph");
    FELOG_REQUIRE(p->window >= 1 && p->window <= 127, "window must be in [1, 127]");
    FELOG_REQUIRE(p->negatives >= 1 && p->negatives <= 20, "negatives must be in [1, 20]");
    FELOG_REQUIRE(p->minibatch_pairs >= 1 && p->minibatch_pairs <= (1 << 24),
                  "minibatch_pairs must be in [1, 2^24]");
    FELOG_REQUIRE(p->chunk_walks >= 0, "chunk_walks must be >= 0");
    FELOG_REQUIRE(std::isfinite(p->lr_start) && std::isfinite(p->lr_end),
                  "learning rates must be finite");
    FELOG_REQUIRE(w->L <= (1 << 23), "walks longer than 2^23 are not supported");
    FELOG_REQUIRE(m->have_noise, "the noise distribution is not set (unigram models need "
                  "felog_model_set_unigram or a first felog_run round)");
    if (m->precision == FELOG_PREC_BF16) {
        FELOG_REQUIRE(p->shared_negatives >= 64 && p->shared_negatives % 64 == 0 &&
                          p->shared_negatives <= (1 << 16),
                      "BF16 models need shared_negatives, a multiple of 64 in [64, 65536]");
        FELOG_REQUIRE(p->minibatch_pairs % 64 == 0 && p->minibatch_pairs <= (1 << 16),
                      "BF16 models need minibatch_pairs a multiple of 64, at most 65536");
    } else {
        FELOG_REQUIRE(p->shared_negatives == 0, "shared negatives need a BF16 model");
    }
}

// FELOG_DEBUG_FAIL_AFTER_MINIBATCHES=N: -1 when unset (or not a number >= 0).
static int64_t fail_after_minibatches()
{
    const char* v = std::getenv("FELOG_DEBUG_FAIL_AFTER_MINIBATCHES");
    if (!v || !*v) return -1;
    char* end = nullptr;
    const long long n = std::strtoll(v, &end, 10);
    return (end && *end == '\0' && n >= 0) ? (int64_t)n : -1;
}

// Trains minibatches [first_mb, first_mb + n_mb) (n_mb < 0: to the end of
// the epoch), stopping after the failure hook's count if it is set.
static void train_range(felog_model* m, const felog_walks* corpus,
                        const felog_train_params* params, int64_t first_mb, int64_t n_mb,
                        felog_train_stats* stats)
{
    const int64_t cut = fail_after_minibatches();
    felog_train_stats st{};
    int64_t n = n_mb;
    if (cut >= 0) n = n_mb < 0 ? cut : std::min(n_mb, cut);
    train_minibatches(*m, *const_cast<felog_walks*>(corpus), *params, first_mb, n, true, &st,
                      nullptr, nullptr, 0, nullptr, nullptr, nullptr, 0, nullptr);
    if (stats) *stats = st;
    if (cut < 0) return;
    const int64_t left = std::max<int64_t>(0, st.minibatches_total - first_mb);
    const int64_t want = n_mb < 0 ? left : std::min(n_mb, left);
    if (want > cut)
        fail(FELOG_EFAULT_INJECTED, "FELOG_DEBUG_FAIL_AFTER_MINIBATCHES=%lld: stopped after "
             "%lld of %lld minibatches", (long long)cut, (long long)st.minibatches,
             (long long)want);
}

felog_status felog_train_epoch(felog_model* m, const felog_walks* corpus,
                               const felog_train_params* params, felog_train_stats* stats)
{
    return guarded([&] {
        check_train_params(m, corpus, params);
        train_range(m, corpus, params, 0, -1, stats);
    });
}

felog_status felog_train_steps(felog_model* m, const felog_walks* corpus,
                               const felog_train_params* params, int64_t first_mb, int64_t n_mb,
                               felog_train_stats* stats)
{
    return guarded([&] {
        check_train_params(m, corpus, params);
        FELOG_REQUIRE(first_mb >= 0 && n_mb >= 0, "minibatch range must be non-negative");
        train_range(m, corpus, params, first_mb, n_mb, stats);
    });
}

felog_status felog_train_delta(felog_model* m, const felog_walks* corpus,
                               const felog_train_params* params, int64_t mb, int32_t* rows_in,
                               float* d_in, int64_t cap_in, int64_t* n_in, int32_t* rows_out,
                               float* d_out, int64_t cap_out, int64_t* n_out, double* loss)
{
    return guarded([&] {
        check_train_params(m, corpus, params);
        NEED(rows_in);
        NEED(d_in);
        NEED(n_in);
        NEED(rows_out);
        NEED(d_out);
        NEED(n_out);
        FELOG_REQUIRE(mb >= 0, "minibatch index must be non-negative");
        felog_train_stats st{};
        train_minibatches(*m, *const_cast<felog_walks*>(corpus), *params, mb, 1, false, &st,
                          rows_in, d_in, cap_in, n_in, rows_out, d_out, cap_out, n_out);
        if (loss) *loss = st.loss;
    });
}

// ---------------------------------------------------------------- feedback
static void check_feedback_params(const felog_feedback_params* p)
{
    NEED(p);
    FELOG_REQUIRE(p->k_s >= 1 && p->k_s <= 64, "k_s must be in [1, 64]");
    FELOG_REQUIRE(p->mode == FELOG_FEEDBACK_MONOTONE || p->mode == FELOG_FEEDBACK_RECOMPUTE_ALL,
                  "unknown feedback mode %d", p->mode);
    FELOG_REQUIRE(!std::isnan(p->mu), "mu must not be NaN");
}

felog_status felog_feedback(felog_model* m, const felog_feedback_params* params,
                            const felog_active* in, felog_active** out, double* psi_host,
                            int64_t psi_cap)
{
    return guarded([&] {
        NEED(m);
        NEED(out);
        *out = nullptr;
        check_feedback_params(params);
        FELOG_REQUIRE(!in || in->g == m->g, "active set belongs to another graph");
        auto a = std::make_unique<felog_active>();
        a->g = m->g;
        const Active* src = params->mode == FELOG_FEEDBACK_RECOMPUTE_ALL ? nullptr : in;
        feedback(*m, *params, src, *a, psi_host, psi_cap);
        *out = a.release();
    });
}

felog_status felog_feedback_noalloc(felog_model* m, const felog_feedback_params* params,
                                    const int32_t* in_nodes_dev, int64_t count,
                                    int32_t* out_nodes_dev, int64_t out_cap, double* psi_dev,
                                    int64_t psi_cap, int64_t* out_count)
{
    return guarded([&] {
        NEED(m);
        NEED(out_count);
        *out_count = 0;
        check_feedback_params(params);
        FELOG_REQUIRE(count >= 0, "count must be >= 0");
        FELOG_REQUIRE(in_nodes_dev || params->mode == FELOG_FEEDBACK_RECOMPUTE_ALL ||
                      count == m->g->n, "in_nodes_dev NULL means all nodes: count must be n");
        feedback_noalloc(*m, *params, in_nodes_dev, count, out_nodes_dev, out_cap, psi_dev,
                         psi_cap, out_count);
    });
}

// --------------------------------------------------------------------- run
// One round's walks and training with the walks written chunk by chunk on the
// context's walk stream: the ids of training chunk k wait for the event of
// walk chunk k only.  *ms_walk is the walk launches' time on their stream.
static void walk_then_train(Model& m, Walks& w, const felog_walk_params& wp,
                            const Active* starts, int64_t n_starts,
                            const felog_train_params& tp, felog_train_stats& ts, double* ms_walk)
{
    Ctx& c = *m.ctx;
    const int64_t chunk = chunk_walks_of(tp);
    FELOG_REQUIRE(chunk >= 1, "chunk_walks must be >= 1");
    plan_valid_columns(w, starts, n_starts, chunk);   // needs no walks; one host sync
    if (!c.walk_stream && !c.single_stream)
        FELOG_HIP(hipStreamCreateWithFlags(&c.walk_stream, hipStreamNonBlocking));
    const hipStream_t ws = c.single_stream ? c.stream : c.walk_stream;
    const int64_t n_chunks = (w.W + chunk - 1) / chunk;
    hipEvent_t t0 = nullptr, t1 = nullptr, after = nullptr;
    FELOG_HIP(hipEventCreate(&t0));
    FELOG_HIP(hipEventCreate(&t1));
    FELOG_HIP(hipEventCreateWithFlags(&after, hipEventDisableTiming));
    w.chunk_ready.assign(n_chunks, nullptr);
    DevBuf cap;
    struct Cleanup {
        Ctx& c;
        Walks& w;
        hipEvent_t* ev[3];
        ~Cleanup()
        {
            // every walk launch has ended before its events and stream go; the
            // stream is not kept, since every stream a process holds takes one
            // of the device's few hardware queues (streams beyond them share
            // queues and lose their concurrency)
            if (c.walk_stream) {
                (void)hipStreamSynchronize(c.walk_stream);
                (void)hipStreamDestroy(c.walk_stream);
                c.walk_stream = nullptr;
            }
            for (hipEvent_t& e : w.chunk_ready)
                if (e) (void)hipEventDestroy(e);
            w.chunk_ready.clear();
            for (hipEvent_t* e : ev)
                if (*e) (void)hipEventDestroy(*e);
        }
    } cleanup{c, w, {&t0, &t1, &after}};
    for (hipEvent_t& e : w.chunk_ready)
        FELOG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    unsigned long long* d_capped = nullptr;
    if (wp.kind != FELOG_WALK_UNIFORM) {
        cap.alloc(&c, sizeof(unsigned long long));
        FELOG_HIP(hipMemsetAsync(cap.ptr, 0, sizeof(unsigned long long), c.stream));
        d_capped = cap.as<unsigned long long>();
    }
    // the walks follow everything already queued for the model (start list, tables)
    FELOG_HIP(hipEventRecord(after, c.stream));
    FELOG_HIP(hipStreamWaitEvent(ws, after, 0));
    FELOG_HIP(hipEventRecord(t0, ws));
    for (int64_t k = 0; k < n_chunks; ++k) {
        const int64_t col0 = k * chunk;
        launch_walk_columns(w, wp, starts, n_starts, col0, std::min(chunk, w.W - col0), ws,
                            d_capped);
        FELOG_HIP(hipEventRecord(w.chunk_ready[k], ws));
    }
    FELOG_HIP(hipEventRecord(t1, ws));
    train_minibatches(m, w, tp, 0, -1, true, &ts, nullptr, nullptr, 0, nullptr, nullptr,
                      nullptr, 0, nullptr);
    FELOG_HIP(hipEventSynchronize(t1));
    float ms = 0.0f;
    FELOG_HIP(hipEventElapsedTime(&ms, t0, t1));
    *ms_walk = ms;
    w.capped = 0;
    if (d_capped) {
        unsigned long long h = 0;
        FELOG_HIP(hipMemcpyAsync(&h, d_capped, sizeof h, hipMemcpyDeviceToHost, c.stream));
        c.sync();
        w.capped = (int64_t)h;
    }
}

felog_status felog_run(felog_model* m, const felog_run_params* p, felog_run_stats* stats)
{
    return guarded([&] {
        NEED(m);
        NEED(p);
        check_walk_params(m->g, &p->walk);
        check_feedback_params(&p->feedback);
        FELOG_REQUIRE(p->max_rounds >= 1 && p->max_rounds <= FELOG_MAX_ROUNDS,
                      "max_rounds must be in [1, %d]", FELOG_MAX_ROUNDS);
        Ctx* c = m->ctx;
        felog_run_stats st{};
        std::unique_ptr<felog_active> act;   // null = all nodes
        int64_t n_active = m->g->n;
        int64_t id_base = 0;
        for (int32_t r = 0; r < p->max_rounds && n_active > 0; ++r) {
            felog_walk_params wp = p->walk;
            wp.id_base = id_base;
            auto w = std::make_unique<felog_walks>();
            w->g = m->g;
            w->L = wp.length;
            w->W = n_active * wp.walks_per_node;
            w->id_base = id_base;
            w->data.alloc(c, sizeof(int32_t) * std::max<int64_t>(w->W * w->L, 1));
            felog_train_stats& ts = st.train[r];
            if (m->have_noise) {
                // Section 5.3's overlap of sampling and training, on one GPU:
                // chunk k + 1 of the round's walks is written on a third stream
                // while the SGNS of chunk k runs.  The walks do not read the
                // tables, so the result is the same as walking first.
                check_train_params(m, w.get(), &p->train);
                walk_then_train(*m, *w, wp, act.get(), n_active, p->train, ts, &st.ms_walk[r]);
            } else {
                // the round-1 unigram noise needs the whole corpus first
                FELOG_HIP(hipEventRecord(c->ev0, c->stream));
                launch_walks(*w, wp, act.get(), n_active);
                FELOG_HIP(hipEventRecord(c->ev1, c->stream));
                c->sync();
                float ms = 0;
                FELOG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
                st.ms_walk[r] = ms;
                DevBuf counts;
                counts.alloc(c, sizeof(uint32_t) * m->g->n);
                launch_corpus_counts(*w, counts.as<uint32_t>());
                build_noise_from_counts(*m, counts.as<uint32_t>());
                c->sync();
                check_train_params(m, w.get(), &p->train);
                train_minibatches(*m, *w, p->train, 0, -1, true, &ts, nullptr, nullptr, 0,
                                  nullptr, nullptr, nullptr, 0, nullptr);
            }
            st.active[r] = n_active;
            st.walks[r] = w->W;
            st.walk_steps[r] = w->n_valid * (int64_t)(w->L - 1);
            id_base += w->W;
            w.reset();
            felog_feedback_params fp = p->feedback;
            fp.round = (uint32_t)r;
            auto next = std::make_unique<felog_active>();
            next->g = m->g;
            FELOG_HIP(hipEventRecord(c->ev0, c->stream));
            const Active* src = fp.mode == FELOG_FEEDBACK_RECOMPUTE_ALL ? nullptr : act.get();
            feedback(*m, fp, src, *next, nullptr, 0);
            FELOG_HIP(hipEventRecord(c->ev1, c->stream));
            c->sync();
            float ms = 0;
            FELOG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
            st.ms_feedback[r] = ms;
            act = std::move(next);
            n_active = act->count;
            st.rounds = r + 1;
        }
        st.final_active = n_active;
        if (stats) *stats = st;
    });
}

}  // extern "C"
