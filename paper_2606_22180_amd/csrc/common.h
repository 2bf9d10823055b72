// Internal declarations of the FeLoG HIP library (gfx950).  Not installed;
// the public interface is include/felog.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <memory>
#include <vector>

#include "felog.h"

namespace felog {

// ---------------------------------------------------------------------------
// Errors: a thread-local message plus the status code returned across the ABI.
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

struct Error {
    felog_status code;
};

[[noreturn]] void fail(felog_status code, const char* fmt, ...);

#define FELOG_HIP(call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            ::felog::fail(e_ == hipErrorOutOfMemory ? FELOG_ENOMEM : FELOG_EDEVICE,  \
                          "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),     \
                          __FILE__, __LINE__);                                       \
    } while (0)

#define FELOG_REQUIRE(cond, ...)                                   \
    do {                                                           \
        if (!(cond)) ::felog::fail(FELOG_EINVAL, __VA_ARGS__);     \
    } while (0)

// ---------------------------------------------------------------------------
// Device memory owned by a context, counted against its HBM budget.
// ---------------------------------------------------------------------------
struct Ctx;

struct DevBuf {
    Ctx* ctx = nullptr;
    void* ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
    DevBuf& operator=(DevBuf&& o) noexcept;
    ~DevBuf() { release(); }
    void alloc(Ctx* c, size_t nbytes);
    void release();
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

constexpr int kIdSets = 3;   // minibatch id buffer sets: ids run kIdSets - 1 minibatches ahead
constexpr int kScanSpanMin = 512;   // fewest touches a block of the SGNS scan passes takes
constexpr int kTimingEvents = 6;   // events per timed minibatch

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t budget = 0;     // 0 = no cap
    uint64_t in_use = 0;
    uint64_t peak = 0;       // largest in_use seen
    int num_cus = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int32_t timing_every = 0;             // time every n-th training launch (0 = off)
    std::vector<hipEvent_t> timing_pool;  // kTimingEvents events per timed minibatch
    // second stream for the table-independent part of later minibatches, and
    // its events: [0] start, [1 + set] ids ready, [1 + kIdSets + set] buffers
    // free, [1 + 2 kIdSets] forward done
    hipStream_t aux = nullptr;
    hipEvent_t pipe_ev[2 + 2 * kIdSets] = {};
    // third stream: walk chunks of a round beside the training of earlier ones
    hipStream_t walk_stream = nullptr;
    // SGNS update path: 0 = the persistent small-minibatch update where it
    // applies, 1 = per-minibatch launches always; workgroups of the persistent
    // launch (0 = one per compute unit)
    int32_t sgns_path = 0;
    int32_t sgns_blocks = 0;
    // every launch on `stream`: the second and third streams are `stream` itself
    bool single_stream = false;
    void make_current() const;
    void sync() const;
    void ensure_aux();
    void release_aux();
};

struct Graph {
    Ctx* ctx = nullptr;
    int32_t n = 0;
    int64_t nnz = 0;
    bool weighted = false;
    DevBuf indptr;    // int64 [n+1]
    DevBuf indices;   // int32 [nnz]
    DevBuf weights;   // float [nnz]   (weighted only; freed once `edges` is built)
    DevBuf edges;     // int2 [nnz]: (index, weight bits) of each entry (weighted only), so
                      // that a node2vec proposal reads one 8-byte record, not two arrays
    DevBuf wmax;      // float [n]     (max weight of each row; 1 when unweighted)
    int64_t isolated = 0;                // nodes without neighbours
};

struct Active {
    Graph* g = nullptr;
    int64_t count = 0;
    DevBuf nodes;     // int32 [count], strictly increasing
};

struct Walks {
    Graph* g = nullptr;
    int64_t W = 0;
    int32_t L = 0;
    int64_t id_base = 0;
    int64_t capped = 0;      // node2vec proposals taken at the attempt cap
    DevBuf data;             // int32 [L][W], step-major, -1 after a walk's end
    // Columns whose walk has at least two nodes (the ones that yield pairs),
    // in column order; built on first use by training.
    bool have_valid = false;
    int64_t n_valid = 0;
    DevBuf valid_cols;       // int32 [n_valid]
    std::vector<int64_t> chunk_valid;   // per chunk of `chunk_for_valid` walks
    int64_t chunk_for_valid = 0;
    // While the walks are still being written on another stream: event c
    // completes when the columns of training chunk c are written (chunks of
    // chunk_for_valid walks).  Training waits for it before reading the chunk.
    std::vector<hipEvent_t> chunk_ready;
};

constexpr int64_t kDefaultChunkWalks = (int64_t)1 << 20;   // walks per training chunk
inline int64_t chunk_walks_of(const felog_train_params& p)
{
    return p.chunk_walks ? p.chunk_walks : kDefaultChunkWalks;
}

// A walk corpus in the FaBC byte format (fabc.hip), in device memory.
constexpr int kFabcMax = 16;   // most symbols a corpus is packed with
struct Packed {
    Graph* g = nullptr;
    int32_t k = 0, L = 0;
    int64_t W = 0, id_base = 0;
    int64_t R = 0;                  // residual positions
    int64_t bytes = 0;
    int32_t symbols[kFabcMax] = {};
    DevBuf buf;                     // the bytes
};

// Buffers of one minibatch's ids and destination sort; kIdSets sets let the
// ids of the next kIdSets - 1 minibatches be computed while one trains.
struct MinibatchBufs {
    DevBuf cnt_in, cnt_out;       // uint32 [n]: touches of each row (0 between minibatches)
    DevBuf off_in, off_out;       // int32 [n]: first entry of each touched row's segment
    DevBuf touch_row;             // int32 [P][K+2]: context, centre, negatives (-1 = skipped)
    DevBuf touch_pos;             // uint32 [P][K+2]: rank of the touch within its row
    DevBuf list_in, list_out;     // int32: touched rows
    DevBuf chunks_in, chunks_out; // int4 per row of <= 16 touches: row, first entry, length, slot
    DevBuf split_in, split_out;   // int4 per chunk of a split row: row, first entry, length, partial
    DevBuf mrows_in, mrows_out;   // int4 per split row: row, first chunk, chunks, list slot
    DevBuf partials;              // per scan block: uint4 (rows, split rows, their chunks), uint64
};

struct Model {
    Ctx* ctx = nullptr;
    Graph* g = nullptr;
    int32_t dim = 0;
    int32_t neg_dist = FELOG_NEG_DEGREE;
    int32_t precision = FELOG_PREC_FP32;
    bool have_noise = false;
    DevBuf tin, tout;             // float [n][d] (the masters of a BF16 model)
    DevBuf bin, bout;             // uint16 [n][d]: BF16 copies (BF16 models), rounded from
                                  // the masters when read out (training rounds as it gathers)
    DevBuf cdf;                   // uint64 [n+1]
    DevBuf guide;                 // int32 [2^guide_bits]
    int32_t guide_bits = 0;
    uint64_t total_weight = 0;
    // minibatch scratch, sized for the largest (pairs, negatives) seen
    bool counters_dirty = false;  // row counters of the id sets may be non-zero
    int64_t cap_pairs = 0;
    int32_t cap_K = 0;
    MinibatchBufs mb[kIdSets];    // by minibatch index mod kIdSets: ids and sort of one minibatch
    DevBuf ent_out;               // int4 [P(K+1)]: (FP64 g, ctx, pair-order key) of each
                                  // out-touch, by row segment
    DevBuf key_in;                // uint32 [P]: pair of each in-row segment position
    DevBuf dinp;                  // float [P][d]: sum_k g_k out[t_k] of each pair (FP64 sum,
                                  // rounded once), by row segment
    DevBuf partial;               // double [chunks of split rows][d]: each chunk's exact sums
    int64_t split_rows_in = 0;    // partial rows reserved for the in-table; the out-table's follow
    DevBuf meta;                  // uint32 [kIdSets][16]: list lengths and counts, by id set
    DevBuf loss_out;              // double [1]
    DevBuf row_totals;            // uint64 [3]: summed touched-list lengths (in, out) and
                                  // out rows touched once
    // small-minibatch update scratch (sgns_small.hip): per launch, each
    // minibatch's touch info, segments, position pairs and counts; per
    // minibatch, the out-touch coefficients, in-row deltas and context copies
    int64_t sm_tmax = 0, sm_G = 0, sm_pairs = 0;
    int32_t sm_dim = 0;
    DevBuf sm_tinfo, sm_segs, sm_spair, sm_meta, sm_gpos, sm_dinp, sm_ctxc;
    // shared-negative (BF16) minibatch scratch
    uint32_t bf_P = 0, bf_M = 0;
    DevBuf bf_ids, bf_C, bf_O, bf_N, bf_Ct, bf_Nt, bf_g0;
    // per-touch update terms and the touches sorted by (table, row): plans of
    // a launch group (small minibatches) or one minibatch with its sort input
    // and radix-sort storage (large ones)
    DevBuf bf_delta, bf_skey, bf_stouch, bf_kin, bf_vin, bf_sort_tmp;
};

// Minibatch schedule of one training call over a corpus.
struct TrainSchedule {
    std::vector<int64_t> chunk_first_mb;   // first global minibatch of each chunk
    std::vector<int64_t> chunk_pairs;
    std::vector<int64_t> chunk_valid_base; // offset of the chunk in valid_cols
    int64_t B = 0;
    int64_t total_pairs = 0;
    int64_t nslices = 0;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplications with the Weyl key schedule.
// ---------------------------------------------------------------------------
struct Rand4 {
    uint32_t v[4];
};

__device__ __forceinline__ Rand4 philox4x32(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint64_t seed)
{
    uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t hi0 = __umulhi(m0, c0), lo0 = m0 * c0;
        uint32_t hi1 = __umulhi(m1, c2), lo1 = m1 * c2;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Rand4{{c0, c1, c2, c3}};
}

// Stream tags (top byte of counter word 3).
constexpr uint32_t kTagWalk = 1u << 24, kTagN2V = 2u << 24, kTagNeg = 3u << 24,
                   kTagInit = 4u << 24, kTagPsi = 5u << 24, kTagSharedNeg = 6u << 24;

// floor(x * m / 2^32): uniform integer below m from 32 random bits.
__device__ __forceinline__ uint32_t scale32(uint32_t x, uint32_t m) { return __umulhi(x, m); }

// ---------------------------------------------------------------------------
// Launch helpers implemented in the .hip files.
// ---------------------------------------------------------------------------
void launch_validate_graph(Graph& g, unsigned long long* d_bad);
void launch_row_wmax(Graph& g);
void build_edge_records(Graph& g);
void launch_walks(Walks& w, const felog_walk_params& p, const Active* starts, int64_t n_starts);
// columns [col0, col0 + ncols) of the corpus on stream s; node2vec adds its
// capped proposals to *d_capped
void launch_walk_columns(Walks& w, const felog_walk_params& p, const Active* starts,
                         int64_t n_starts, int64_t col0, int64_t ncols, hipStream_t s,
                         unsigned long long* d_capped);
void launch_valid_columns(Walks& w, int64_t chunk);
// the same columns and counts from the start list, before the walks exist
void plan_valid_columns(Walks& w, const Active* starts, int64_t n_starts, int64_t chunk);
void launch_init_tables(Model& m, uint64_t seed);
void build_noise_from_counts(Model& m, const uint32_t* d_counts);   // counts in device memory
void set_noise_cdf(Model& m, const uint64_t* host_cdf);   // a saved table, checked
void launch_degree_counts(Graph& g, uint32_t* d_counts);
void launch_corpus_counts(const Walks& w, uint32_t* d_counts);
void train_minibatches(Model& m, const Walks& w, const felog_train_params& p, int64_t first_mb,
                       int64_t n_mb, bool apply, felog_train_stats* stats,
                       int32_t* rows_in, float* d_in, int64_t cap_in, int64_t* n_in,
                       int32_t* rows_out, float* d_out, int64_t cap_out, int64_t* n_out);
int64_t count_minibatches(Walks& w, const felog_train_params& p, int64_t* total_pairs);
void model_alloc_update_state(Model& m);   // row counters, offsets, minibatch counters
void fabc_profile(const Walks& w, int32_t k_max, int32_t* k, int32_t* symbols,
                  uint64_t* counts, int32_t* n_ranked, uint64_t* total);
void fabc_pack(const Walks& w, int32_t k, const int32_t* symbols, Packed& p, double* ms);
void fabc_from_host(Graph& g, const void* host, int64_t bytes, Packed& p);
void fabc_unpack(const Packed& p, Walks& w, double* ms);
void train_minibatches_bf16(Model& m, Walks& w, const felog_train_params& p,
                            const TrainSchedule& sch, const int32_t* d_slices, int64_t first_mb,
                            int64_t end, float* cap_in, float* cap_out, felog_train_stats* stats);
void bf16_refresh_all(Model& m);
// The persistent small-minibatch FP32 update (P (K + 2) <= 8192 touches).
bool small_path_applies(const Model& m, const felog_train_params& p);
void train_minibatches_small(Model& m, Walks& w, const felog_train_params& p,
                             const TrainSchedule& sch, const int32_t* d_slices, int64_t first_mb,
                             int64_t end, felog_train_stats* stats);
void launch_loss_reduce(const double* part, int64_t n, double* out, hipStream_t s);
int64_t small_minibatches_per_launch();
// touches per minibatch, P (K + 2), up to which the persistent update applies
constexpr int kSmallMaxTouches = 8192;
// jobs whose minibatches one shared persistent launch can carry
constexpr int kMaxBatchJobs = 8;

// The schedule and pair slices of a training call over a corpus.
TrainSchedule train_schedule(Walks& w, const felog_train_params& p);
std::vector<int32_t> train_slices(int32_t L, int32_t window);

// Training calls of several models in shared persistent launches (serving):
// each launch plans and updates the next launch group of up to
// kMaxBatchJobs jobs of equal d and K, phase by phase together.
struct SmallJob;
struct SmallJobDeleter {
    void operator()(SmallJob* j) const;
};
using SmallJobPtr = std::unique_ptr<SmallJob, SmallJobDeleter>;
struct SmallBatchCtl {
    DevBuf words;        // barrier flags and the abort flag of the shared launches
    uint32_t epoch = 0;  // barriers passed so far
    int nblocks = 0;
};
bool small_job_fits(const Model& m, const felog_train_params& p);
// Prepares the model's buffers and the call's descriptors (on the model's
// stream, then waits for it); nblocks is the grid of the shared launches.
SmallJobPtr small_job_begin(Model& m, Walks& w, const felog_train_params& p, int nblocks);
int small_job_dim(const SmallJob& j);
int small_job_negatives(const SmallJob& j);
bool small_job_done(const SmallJob& j);
int small_update_blocks(const Ctx& c, int D, int K);
void small_batch_init(SmallBatchCtl& ctl, Ctx& c, int nblocks);
void small_jobs_step(const std::vector<SmallJob*>& jobs, SmallBatchCtl& ctl, hipStream_t s);
bool small_batch_aborted(SmallBatchCtl& ctl, hipStream_t s);   // waits for the stream
void small_job_end(SmallJob& j, hipStream_t s, felog_train_stats* stats);   // waits too
uint64_t small_path_bytes(int64_t P, int K, int d, int64_t B, int num_cus);
void feedback(Model& m, const felog_feedback_params& p, const Active* in, Active& out,
              double* psi_host, int64_t psi_cap);
// The feedback step with no device allocation: Psi into the caller's psi[],
// the kept ids into out_nodes[]; scratch is a fixed per-device array whose
// address noalloc_scratch_init (called once per device, from context
// creation) looks up.
void noalloc_scratch_init(int device);
void feedback_noalloc(Model& m, const felog_feedback_params& p, const int32_t* in_nodes,
                      int64_t count, int32_t* out_nodes, int64_t out_cap, double* psi,
                      int64_t psi_cap, int64_t* out_count);
// Order-preserving compaction of nodes[i] where flags[i] != 0; returns the count.
int64_t compact_nodes(Ctx& ctx, const int32_t* d_nodes, const uint8_t* d_flags, int64_t count,
                      DevBuf& out);

}  // namespace felog
