/*
 * felog.h -- C ABI of the FeLoG hot path on one AMD Instinct MI355X (gfx950).
 *
 * The method (FeLoG, arxiv 2606.22180, Section 5.1 and Algorithm 1): generate
 * random walks from the active nodes (Sample), train skip-gram with negative
 * sampling on them (Train, Eq. (1)-(2)), score each active node by the mean
 * cosine between its embedding and a subsample of its neighbours' (Psi,
 * Eq. (4)), keep the nodes with Psi < mu (Eq. (5)), and repeat.
 *
 * Conventions
 *  - Every call returns felog_status: FELOG_OK (0) or a negative error code.
 *    felog_last_error() returns a message for the calling thread's last error;
 *    it stays valid until that thread's next felog_* call.  No C++ exception
 *    crosses this boundary.
 *  - Handles are opaque.  Each *_create / *_generate / *_load has a matching
 *    *_destroy; *_destroy(NULL) is a no-op.  The library owns every device
 *    buffer behind a handle and frees it in *_destroy.
 *  - Host pointers passed in are read during the call and never retained.
 *    Host output buffers are written during the call and are owned by the
 *    caller.  Output buffers smaller than the result give FELOG_EINVAL.
 *  - A context is bound to one device and one HIP stream.  Calls enqueue work
 *    on that stream and return after it completes, unless documented otherwise.
 *    A context and the handles made from it are used by one thread at a time.
 *  - Node ids are int32; sizes and counts are int64.
 *  - Device work runs in hand-written HIP kernels; no call falls back to the
 *    host for any step of the method.
 */
#ifndef FELOG_H
#define FELOG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t felog_status;

enum {
    FELOG_OK = 0,
    FELOG_EINVAL = -1,        /* bad argument, malformed graph, buffer too small   */
    FELOG_ENOMEM = -2,        /* device allocation failed or HBM budget exceeded   */
    FELOG_EDEVICE = -3,       /* a HIP call failed                                 */
    FELOG_ESTATE = -4,        /* handle in the wrong state for this call           */
    FELOG_EUNSUPPORTED = -5,  /* valid request this build does not implement        */
    FELOG_EIO = -6,           /* a file could not be opened, read or written        */
    FELOG_EFAULT_INJECTED = -7, /* the training call stopped where the debug hook
                                   FELOG_DEBUG_FAIL_AFTER_MINIBATCHES asked it to    */
};

typedef struct felog_ctx felog_ctx;
typedef struct felog_graph felog_graph;
typedef struct felog_walks felog_walks;
typedef struct felog_packed felog_packed;
typedef struct felog_active felog_active;
typedef struct felog_model felog_model;

/* ------------------------------------------------------------------------- */
/* Context                                                                    */
/* ------------------------------------------------------------------------- */

/* Bind a context to HIP device `device` and stream `hip_stream` (a hipStream_t,
 * or NULL for the null stream).  `hbm_budget_bytes` caps the device memory the
 * context may hold at once (0 = no cap); an allocation beyond it fails with
 * FELOG_ENOMEM. */
felog_status felog_ctx_create(int device, void* hip_stream, uint64_t hbm_budget_bytes,
                              felog_ctx** out);
/* Every object created on the context (graphs and what is made from them)
 * must be destroyed before the context. */
void felog_ctx_destroy(felog_ctx* ctx);

/* Device bytes currently held by handles of this context. */
felog_status felog_ctx_bytes_in_use(const felog_ctx* ctx, uint64_t* bytes);

/* Kernel timing: with every > 0, training brackets every `every`-th forward
 * and apply launch with HIP events on the context's stream and reports their
 * summed durations in felog_train_stats (0 = off, the default). */
felog_status felog_ctx_set_timing(felog_ctx* ctx, int32_t every);

/* SGNS update path of the FP32 form.  path 0 (the default): minibatches of
 * P (K + 2) <= 8192 touches (and K <= 14 at d = 64) run as plan launches (ids and a sort of each
 * minibatch's touches by row, many minibatches per launch) and one persistent
 * cooperative update launch per group of minibatches; larger ones run
 * per-minibatch launches.  path 1: per-minibatch launches always.  Both give
 * bit-identical tables.  blocks: workgroups of the persistent launch (0 = the
 * default, 64; capped at what can be resident at once).  With timing on
 * (felog_ctx_set_timing), every plan and update launch of path 0 is timed.
 * Errors: path not 0 or 1, blocks outside [0, 65536]. */
felog_status felog_ctx_set_sgns_path(felog_ctx* ctx, int32_t path, int32_t blocks);

/* on = 1: every launch of the context goes to its one stream.  The plans of
 * later minibatches, the ids of the large-minibatch path and the walks that
 * felog_run writes beside training then run in issue order after the
 * launches they would overlap; results are unchanged.  For tools that follow
 * one stream (profilers, stream capture).  on = 0 (the default) restores the
 * second and third streams.  Waits for the context's second stream first.
 * Errors: on not 0 or 1. */
felog_status felog_ctx_set_single_stream(felog_ctx* ctx, int32_t on);

/* Message for the calling thread's last failed call ("" if none). */
const char* felog_last_error(void);

/* ------------------------------------------------------------------------- */
/* Graph (Table 1: G = (V, E), undirected, unweighted; weighted for node2vec)  */
/* ------------------------------------------------------------------------- */

/* Upload a symmetric CSR graph.  indptr[n_nodes+1] (int64, indptr[0] = 0,
 * indptr[n] = nnz, non-decreasing), indices[nnz] (int32 in [0, n), strictly
 * increasing within each row, no self loops), weights[nnz] (float32 > 0, or
 * NULL for an unweighted graph).  The graph must be symmetric (v in N(u) iff
 * u in N(v)) with equal weights on both directions; a graph that is not gives
 * FELOG_EINVAL with a message naming the first offending row.  The caller's
 * arrays are copied; the call returns after the upload and the checks.  On the
 * device a weighted graph keeps 8 bytes per entry (index and weight side by
 * side, for node2vec proposals) besides the indices; an unweighted one 4. */
felog_status felog_graph_load_csr(felog_ctx* ctx, int32_t n_nodes, int64_t nnz,
                                  const int64_t* indptr, const int32_t* indices,
                                  const float* weights, felog_graph** out);
void felog_graph_destroy(felog_graph* g);
felog_status felog_graph_info(const felog_graph* g, int32_t* n_nodes, int64_t* nnz,
                              int32_t* weighted);

/* ------------------------------------------------------------------------- */
/* Active node sets (V_a of Algorithm 1), sorted ascending on the device        */
/* ------------------------------------------------------------------------- */

/* Copy a strictly increasing list of node ids to the device. */
felog_status felog_active_from_host(felog_graph* g, const int32_t* sorted_nodes, int64_t count,
                                    felog_active** out);
/* All nodes 0..n-1 (V_a at the first round). */
felog_status felog_active_all(felog_graph* g, felog_active** out);
felog_status felog_active_count(const felog_active* a, int64_t* count);
/* Copy the list to host memory nodes[cap]; *count receives its length. */
felog_status felog_active_read(const felog_active* a, int32_t* nodes, int64_t cap,
                               int64_t* count);
void felog_active_destroy(felog_active* a);

/* ------------------------------------------------------------------------- */
/* Sample: random walks (Section 2 "Sampling process"; Section 5.1 Sample)      */
/* ------------------------------------------------------------------------- */

enum { FELOG_WALK_UNIFORM = 0, FELOG_WALK_NODE2VEC = 1 };

typedef struct felog_walk_params {
    int32_t kind;             /* FELOG_WALK_UNIFORM or FELOG_WALK_NODE2VEC        */
    int32_t walks_per_node;   /* r >= 1                                           */
    int32_t length;           /* L >= 1 nodes per walk, start included            */
    float p, q;               /* node2vec return / in-out parameters (> 0)         */
    uint64_t seed;            /* Philox key                                        */
    int64_t id_base;          /* id of the first walk (walk ids key the RNG)       */
} felog_walk_params;

/* Generate r walks per start node.  Walk i (0 <= i < r * |starts|) has id
 * id_base + i and starts at starts[i mod |starts|] (starts = NULL: all nodes).
 * Uniform: transition t moves to neighbour floor(x0 * deg / 2^32), x0 from
 * Philox(key = seed, counter = (id low, id high, t, 1 << 24)).  node2vec:
 * rejection sampling of w(v,x) * alpha(t,x) with alpha = 1/p, 1, 1/q (return,
 * common neighbour, outward); attempt a uses counter (id low, id high, t,
 * 2 << 24 | a).
 * A start node without neighbours gives a one-node walk.  The walks stay on
 * the device. */
felog_status felog_walks_generate(felog_graph* g, const felog_walk_params* params,
                                  const felog_active* starts, felog_walks** out);
felog_status felog_walks_info(const felog_walks* w, int64_t* n_walks, int32_t* length,
                              int64_t* id_base);
/* Copy walks to host memory as walk-major int32 [n_walks][length], -1 after a
 * walk's end.  cap is the element capacity of `walks`. */
felog_status felog_walks_read(const felog_walks* w, int32_t* walks, int64_t cap);
/* Walks first .. first + count - 1 only, walk-major int32 [count][L] into host
 * memory (cap ints); EINVAL if the range leaves [0, W). */
felog_status felog_walks_read_range(const felog_walks* w, int64_t first, int64_t count,
                                    int32_t* walks, int64_t cap);
/* Number of node2vec proposals that hit the attempt cap (expected 0). */
felog_status felog_walks_capped(const felog_walks* w, int64_t* capped);
void felog_walks_destroy(felog_walks* w);

/* ------------------------------------------------------------------------- */
/* Walk-corpus codec (FaBC: frequency-aware bitmap compression, Section 5.2.2, */
/* Eq. (6)-(8)).  Symbols are node ids and -1, the padding after an isolated */
/* start's only node.                                                         */
/* ------------------------------------------------------------------------- */

#define FELOG_FABC_MAX_SYMBOLS 16

/* Profile a corpus: every symbol's share p of the W*L positions, ranked by
 * count (descending) then symbol (ascending); then the target set of Eq. (8):
 * k grows while p(k+1) >= c + 0.1 g(k), with c = 1/L + 1/32 and
 * g(k) = (1 - F_k) + k c (Eq. (7), F_k the top k's share), evaluated in FP64
 * as written, k <= k_max <= 16.  Outputs: *k; the first *n_ranked (<= k_max)
 * ranked symbols and their counts in symbols[k_max] / counts[k_max] (host
 * buffers; fewer when fewer symbols occur); *total = W*L. */
felog_status felog_fabc_profile(const felog_walks* w, int32_t k_max, int32_t* k,
                                int32_t* symbols, uint64_t* counts, int32_t* n_ranked,
                                uint64_t* total);

/* Pack a corpus with the given k <= 16 distinct symbols (in [-1, n)), on the
 * device.  Byte format (little endian):
 *   header    u32 0x43426146, u32 k, u32 L, u32 0, u64 W, i64 id_base   32 B
 *   symbols   i32[k]
 *   bitmaps   u8[k][ceil(L/8)][W]: bit j%8 of byte j/8 of symbol b's bitmap
 *             of walk w is set iff position j of walk w holds symbol b
 *   padding   zero bytes to a multiple of 8
 *   offsets   u64[ceil(W/256)]: residual positions before walk 256 i
 *   residuals i32[R]: every other position, walk by walk, position ascending
 * Its size is Eq. (6) with the symbols stored once per corpus, plus the
 * header, padding and offsets.  ms (nullable, double[2]): device time of the
 * counting and the writing launches. */
felog_status felog_walks_pack(const felog_walks* w, int32_t k, const int32_t* symbols,
                              felog_packed** out, double* ms);
/* Sizes: total bytes, k, walks W, length L, residual positions R (each nullable). */
felog_status felog_packed_info(const felog_packed* p, int64_t* bytes, int32_t* k,
                               int64_t* n_walks, int32_t* length, int64_t* residuals);
/* Copy the packed bytes to host memory (cap >= bytes). */
felog_status felog_packed_read(const felog_packed* p, void* host, int64_t cap);
/* Upload packed bytes for a graph.  The header, the symbols (in [-1, n),
 * distinct) and the size are checked here; the bitmaps, offsets and residuals
 * when unpacking. */
felog_status felog_packed_from_host(felog_graph* g, const void* host, int64_t bytes,
                                    felog_packed** out);
/* Unpack into a new corpus on the device (same walks, length and walk ids as
 * the packed one).  A corpus whose bitmaps overlap, whose offsets disagree
 * with its bitmaps or whose residuals are missing or outside [-1, n) gives
 * FELOG_EINVAL.  ms (nullable): device time of the unpacking launch. */
felog_status felog_packed_unpack(const felog_packed* p, felog_walks** out, double* ms);
void felog_packed_destroy(felog_packed* p);

/* ------------------------------------------------------------------------- */
/* Model: embedding tables phi_in, phi_out (Eq. (2)) and the noise distribution */
/* ------------------------------------------------------------------------- */

enum { FELOG_NEG_DEGREE = 0, FELOG_NEG_UNIGRAM = 1 };
enum { FELOG_TABLE_IN = 0, FELOG_TABLE_OUT = 1 };
enum { FELOG_PREC_FP32 = 0, FELOG_PREC_BF16 = 1 };

typedef struct felog_model_params {
    int32_t dim;              /* d; 64, 128 or 256                                */
    int32_t neg_dist;         /* FELOG_NEG_DEGREE or FELOG_NEG_UNIGRAM             */
    uint64_t seed;            /* Philox key of the initial in-table                */
    int32_t precision;        /* FELOG_PREC_FP32: FP32 tables, per-pair negatives;
                                 FELOG_PREC_BF16: FP32 master tables plus BF16
                                 copies read by shared-negative MFMA training      */
} felog_model_params;

/* Create FP32 tables [n][d]: in[v][c] = ((x >> 8) * 2^-24 - 0.5) / d with x
 * word c mod 4 of Philox(key = seed, counter = (v low, v high, c / 4, 4 << 24));
 * out = 0.
 * With FELOG_NEG_DEGREE the noise distribution is degree^0.75 at once; with
 * FELOG_NEG_UNIGRAM it is set from the first corpus passed to training. */
felog_status felog_model_create(felog_graph* g, const felog_model_params* params,
                                felog_model** out);
void felog_model_destroy(felog_model* m);

/* Set the noise distribution Pn(u) ~ c_u^0.75 from the node counts of a walk
 * corpus (the unigram distribution).  Weight of u: floor(2^16 * sqrt(c) *
 * sqrt(sqrt(c))) in IEEE double; a draw maps 64 random bits x to
 * floor(x * T / 2^64) and returns the node whose cumulative-weight interval
 * holds it. */
felog_status felog_model_set_unigram(felog_model* m, const felog_walks* corpus);
/* Copy the integer cumulative weights cdf[n+1] (uint64) to host memory. */
felog_status felog_model_read_cdf(const felog_model* m, uint64_t* cdf, int64_t cap);

/* Copy a BF16 model's BF16 copy of a table (bit patterns, row-major [n][d]);
 * every row equals its FP32 master rounded to nearest even. */
felog_status felog_embeddings_read_bf16(const felog_model* m, int32_t which, uint16_t* host,
                                        int64_t cap);
/* Copy a table (FELOG_TABLE_IN / FELOG_TABLE_OUT) as row-major float32 [n][d]
 * (the FP32 masters of a BF16 model). */
felog_status felog_embeddings_read(const felog_model* m, int32_t which, float* host, int64_t cap);
/* Same into device memory (e.g. a torch tensor's data pointer) on the context's stream. */
felog_status felog_embeddings_read_dev(const felog_model* m, int32_t which, void* dev,
                                       int64_t cap);
/* Shape of a model: nodes, dimension, noise distribution, precision (each
 * pointer may be NULL). */
felog_status felog_model_info(const felog_model* m, int32_t* n, int32_t* dim, int32_t* neg_dist,
                              int32_t* precision);

/* Persist(S, V) of the deployment view (Section 5.4), the V half: the model's
 * state to a file and back, so that Algorithm 1 can resume at a round.  (The
 * S half is the walk corpus in the FaBC format: felog_walks_pack and
 * felog_packed_read give its bytes, felog_packed_from_host takes them back.)
 *
 * File layout, little endian:
 *   header 64 B  u32 magic 0x4D4C6546 ("FeLM"), u32 version 1, i32 n, i32 d,
 *                i32 neg_dist, i32 precision, u32 round, u32 flags (bit 0:
 *                noise table present, bit 1: active list present),
 *                i64 walk_id_base, i64 active count, u64 graph nnz, u64 0
 *   in table     f32 [n][d] (the FP32 masters of a BF16 model)
 *   out table    f32 [n][d]
 *   noise        u64 [n + 1] cumulative weights, when flags bit 0
 *   active list  i32 [count], strictly increasing, when flags bit 1
 * `round` and `walk_id_base` are the caller's round metadata (the next round
 * of Algorithm 1 and the first walk id it uses); they are stored as given.
 * A BF16 model's copies are rounded from the restored masters when read.
 * The file is written whole or the call fails with FELOG_EIO (a partial file
 * may remain); loading checks the header against the graph (n, nnz), the
 * file size, the noise table (starts at 0, non-decreasing, positive total)
 * and the active list (sorted, in range) and fails with FELOG_EINVAL or
 * FELOG_EIO. */
typedef struct felog_checkpoint_meta {
    uint32_t round;
    int64_t walk_id_base;
} felog_checkpoint_meta;

/* active and meta may be NULL (no list; round 0, id base 0). */
felog_status felog_model_save(const felog_model* m, const felog_active* active,
                              const felog_checkpoint_meta* meta, const char* path);
/* *out: a new model on graph g.  *active (when active is not NULL): the saved
 * list, or NULL if the file has none.  meta (nullable) receives the round
 * metadata. */
felog_status felog_model_load(felog_graph* g, const char* path, felog_model** out,
                              felog_active** active, felog_checkpoint_meta* meta);

/* Re-initialise the tables as felog_model_create does (in from `seed`,
 * out = 0); a unigram noise distribution is cleared so that the next
 * felog_run sets it again from its first round. */
felog_status felog_model_reset(felog_model* m, uint64_t seed);
/* Overwrite a table from host memory (count = n * d floats). */
felog_status felog_embeddings_write(felog_model* m, int32_t which, const float* host,
                                    int64_t count);

/* ------------------------------------------------------------------------- */
/* Train: skip-gram with negative sampling (Eq. (1), Eq. (2))                  */
/* ------------------------------------------------------------------------- */

typedef struct felog_train_params {
    int32_t window;           /* w: offsets i in [-w, w] \ {0}                     */
    int32_t negatives;        /* K negatives per pair                              */
    float lr_start, lr_end;   /* linear decay over the call's minibatches          */
    int64_t minibatch_pairs;  /* P pairs per minibatch                             */
    int64_t chunk_walks;      /* pairs are ordered within chunks of this many walks
                                 (0 = 2^20)                                        */
    uint64_t seed;            /* Philox key of the negative draws                  */
    int32_t shared_negatives; /* BF16 models: M negatives shared by the pairs of a
                                 minibatch (P and M multiples of 64); 0 for FP32   */
} felog_train_params;

typedef struct felog_train_stats {
    int64_t minibatches;      /* minibatches run by the call                       */
    int64_t pairs;            /* (context, centre) pairs trained                   */
    int64_t minibatches_total;/* minibatches in the whole corpus                   */
    double loss;              /* sum over the call's pairs of -log sigma(s0)
                                 - sum_k log sigma(-s_k), FP64                     */
    double ms;                /* device time of the call                           */
    int64_t rows_in;          /* sum over minibatches of distinct in-rows updated  */
    int64_t rows_out;         /* sum over minibatches of distinct out-rows updated */
    int64_t timed_launches;   /* forward (and apply) launches timed with events    */
    double ms_forward;        /* summed duration of the timed forward launches     */
    double ms_apply;          /* summed duration of the timed apply launches       */
    double ms_prep;           /* summed duration of the timed id / rank / offset   */
                              /* launches that precede each timed forward          */
    double ms_apply_first;    /* summed duration of the first of the timed apply
                                 launches (out rows, chunks of split rows)         */
    int64_t rows_out_single;  /* of rows_out, the rows touched once in their
                                 minibatch (updated by the forward launch)          */
    int32_t path;             /* update path the call took: 0 per-minibatch launches,
                                 1 the persistent small-minibatch update             */
    int32_t update_blocks;    /* path 1: workgroups of the persistent launch         */
    int64_t timed_minibatches;/* path 1: minibatches covered by the timed launches   */
    double ms_update;         /* path 1: summed duration of the timed persistent
                                 update launches (ms_prep: their plan launches)      */
    double us_phase[4];       /* path 1 with timing on: mean time per minibatch and
                                 workgroup of the update's forward phase, its first
                                 grid barrier, the apply phase and the second barrier
                                 (us, device wall clock; a phase ends when every wave
                                 of the workgroup reaches the barrier, a barrier when
                                 the workgroup leaves it)                            */
} felog_train_stats;

/* One Train() call: every minibatch of the corpus in order.  Pairs: within each
 * chunk, centre position j, then offset slot (i = -w..-1, 1..w), then walk; a
 * minibatch is the next P pairs of the chunk.  Every pair reads the tables as
 * they stand at the minibatch's start; the minibatch's deltas are summed per
 * row and then added:
 *   g0 = lr (1 - sigma(in[c].out[t0])),  gk = -lr sigma(in[c].out[tk])
 *   delta in[c] += sum_k gk out[tk],   delta out[tk] += gk in[c].
 * Negative k of a pair uses words 2(k mod 2), 2(k mod 2)+1 (low, high) of
 * Philox(key = seed, counter = (walk id low, walk id high, j << 8 | slot,
 * 3 << 24 | k / 2)); a negative equal to the centre is skipped.  lr for minibatch b of B: lr_start - (lr_start - lr_end) b / (B-1).
 * Arithmetic: dots, sigma and the coefficients in FP64 over the FP32 entries;
 * a row's terms summed in FP64 (in pair order for rows of at most 16 touches,
 * rounded onto a grid on which FP64 addition is exact for longer rows) and
 * added to the FP32 entry with one rounding; a row touched once takes its one
 * term the same way.  The tables are identical on both update paths and from
 * run to run. */
/* Failure hook (the library's only environment variable): when
 * FELOG_DEBUG_FAIL_AFTER_MINIBATCHES=N (N >= 0) is set, felog_train_epoch and
 * felog_train_steps train at most the first N minibatches of their range and,
 * if the range holds more, return FELOG_EFAULT_INJECTED with the tables as
 * those N minibatches left them (stats, when given, describe those N).  It
 * stands in for a failure in the middle of a round, so that recovery from a
 * checkpoint (felog_model_save / felog_model_load) can be tested. */
felog_status felog_train_epoch(felog_model* m, const felog_walks* corpus,
                               const felog_train_params* params, felog_train_stats* stats);
/* BF16 models (shared negatives, not in the paper; a systems form of Eq. (2)):
 * minibatch b of a corpus whose first walk id is B draws M negatives, m-th from
 * words 2(m mod 2), 2(m mod 2)+1 of Philox(key = seed, counter = (b, low 32 bits
 * of B, m / 2, 6 << 24)); every (pair, negative) term has weight K / M, terms
 * whose negative equals the pair's centre are dropped.  With C = BF16 rows of
 * in[ctx], N = BF16 rows of out[neg], O = BF16 rows of out[ctr]:
 *   S = C N^T (MFMA, FP32 accumulation),  G = bf16(-lr (K/M) sigma(S) o mask),
 *   delta in[ctx] += G N + g0 O,  delta out[neg] += G^T C,  delta out[ctr] += g0 C,
 * g0 = lr (1 - sigma(rowwise C.O)); sigma of S from the hardware exp2, rcp and
 * log2 (a few FP32 ulps before the BF16 rounding of G).  Each touch's term is
 * FP32; every touched row sums its terms in FP64 in touch order (contexts,
 * then centres, then negatives) and the FP32 master takes the sum with one
 * rounding, so the tables are bit-reproducible.  The BF16 rows of a
 * minibatch are its masters at the minibatch's start, rounded to nearest
 * even. */

/* Minibatches [first_mb, first_mb + n_mb) of the same schedule (the tables must
 * hold the state at the start of first_mb). */
felog_status felog_train_steps(felog_model* m, const felog_walks* corpus,
                               const felog_train_params* params, int64_t first_mb,
                               int64_t n_mb, felog_train_stats* stats);
/* The summed deltas of minibatch `mb` without applying them (for checking one
 * step).  rows_in / rows_out receive the touched rows (any order) and
 * d_in / d_out their FP32 deltas, row-major [count][d]; capacities in rows. */
felog_status felog_train_delta(felog_model* m, const felog_walks* corpus,
                               const felog_train_params* params, int64_t mb,
                               int32_t* rows_in, float* d_in, int64_t cap_in, int64_t* n_in,
                               int32_t* rows_out, float* d_out, int64_t cap_out,
                               int64_t* n_out, double* loss);

/* ------------------------------------------------------------------------- */
/* Feedback: Psi (Eq. (4)) and the next active set (Eq. (5))                 */
/* ------------------------------------------------------------------------- */

enum { FELOG_FEEDBACK_MONOTONE = 0, FELOG_FEEDBACK_RECOMPUTE_ALL = 1 };

typedef struct felog_feedback_params {
    double mu;                /* keep v when Psi(v) < mu                           */
    int32_t k_s;              /* neighbour subsample size (1..64)                  */
    int32_t mode;             /* MONOTONE: score `in`; RECOMPUTE_ALL: score all V  */
    uint64_t seed;            /* Philox key of the neighbour subsets               */
    uint32_t round;           /* round number, part of the subset counter          */
} felog_feedback_params;

/* Psi(v) = mean over a neighbour subset of cos(in[v], in[u]): all neighbours
 * when deg(v) <= k_s, else k_s distinct ones by Floyd's algorithm with draw m
 * from Philox(key = seed, counter = (v, round, m / 4, 5 << 24)) word m mod 4.
 * FP64 products and sums.  *out receives {v : Psi(v) < mu}, sorted; nodes
 * without neighbours are never kept.  psi_host (nullable) receives Psi of the
 * scored nodes in list order (NaN for nodes without neighbours). */
felog_status felog_feedback(felog_model* m, const felog_feedback_params* params,
                            const felog_active* in, felog_active** out, double* psi_host,
                            int64_t psi_cap);

/* The feedback step with no device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same scores and decisions as
 * felog_feedback.  All buffers are the caller's device memory:
 *   in_nodes_dev   int32 [count], strictly increasing node ids (checked), the
 *                  scored list of the MONOTONE mode; NULL = all nodes (count
 *                  must then be n).  RECOMPUTE_ALL ignores it and scores all n.
 *   out_nodes_dev  int32 [out_cap]: the kept nodes {v : Psi(v) < mu}, in list
 *                  order; out_cap >= the number of scored nodes.
 *   psi_dev        double [psi_cap]: Psi of every scored node, in list order
 *                  (NaN for nodes without neighbours); psi_cap >= scored.
 *   *out_count     (host) number of kept nodes.
 * At most 2^24 nodes are scored per call (FELOG_EINVAL beyond).  The only
 * scratch is a fixed array of about 33 KB that each device holds from its
 * first context until the process ends; calls that overlap on one device
 * share it and race, so they must be serialised (one stream, or one call at
 * a time).  Work runs on the model's context stream; the call returns after
 * it completes. */
felog_status felog_feedback_noalloc(felog_model* m, const felog_feedback_params* params,
                                    const int32_t* in_nodes_dev, int64_t count,
                                    int32_t* out_nodes_dev, int64_t out_cap, double* psi_dev,
                                    int64_t psi_cap, int64_t* out_count);

/* ------------------------------------------------------------------------- */
/* Algorithm 1 end to end                                                      */
/* ------------------------------------------------------------------------- */

typedef struct felog_run_params {
    felog_walk_params walk;        /* id_base is ignored: rounds number walks on */
    felog_train_params train;
    felog_feedback_params feedback;/* round is set by the loop                   */
    int32_t max_rounds;            /* stop after this many rounds (>= 1)         */
} felog_run_params;

#define FELOG_MAX_ROUNDS 64

typedef struct felog_run_stats {
    int32_t rounds;
    int64_t active[FELOG_MAX_ROUNDS];      /* |V_a| at the start of each round   */
    int64_t walks[FELOG_MAX_ROUNDS];
    int64_t walk_steps[FELOG_MAX_ROUNDS];  /* transitions taken                  */
    double ms_walk[FELOG_MAX_ROUNDS];      /* walk launches, on their stream     */
    double ms_feedback[FELOG_MAX_ROUNDS];
    felog_train_stats train[FELOG_MAX_ROUNDS];
    int64_t final_active;                  /* |V_a| after the last round         */
} felog_run_stats;

/* Algorithm 1: V_a = V; while V_a is not empty and fewer than max_rounds rounds
 * ran: walks from V_a, one training call over them (the unigram noise
 * distribution is set from the first round's corpus if the model asks for it),
 * feedback on V_a (or on V in RECOMPUTE_ALL mode), V_a = result.
 * Sampling overlaps training (Section 5.3): once the noise distribution is
 * set, a round's walks are written chunk by chunk (train.chunk_walks walks,
 * default 2^20) on a stream the call creates and releases, beside the
 * training, which reads chunk k as soon as its walks are written.  The
 * results are those of walking first.  Calls on one model must not overlap. */
felog_status felog_run(felog_model* m, const felog_run_params* params, felog_run_stats* stats);

/* ------------------------------------------------------------------------- */
/* Serving: continuous admission of embedding jobs under an HBM budget       */
/* (a systems form, not in the paper)                                        */
/* ------------------------------------------------------------------------- */

typedef struct felog_server felog_server;

typedef struct felog_server_params {
    int32_t slots;            /* jobs on the device at once (1..4; 1..3 when shared)  */
    int64_t minibatch_pairs;  /* largest P of a job; a job on n nodes uses            */
                              /* min(minibatch_pairs, the next power of two >= n):    */
                              /* summed minibatch updates diverge once P is large     */
                              /* next to n (rows touched hundreds of times per step)  */
    int32_t negatives;        /* K for every job                                       */
    float lr_start, lr_end;   /* learning-rate decay over each job's epoch             */
    int32_t update_mode;      /* FELOG_SERVE_*: how the jobs' SGNS minibatches run     */
} felog_server_params;

/* Update modes of a server (the tables are the same in every mode):
 *   FELOG_SERVE_LAUNCHES (0, the default): each job's per-minibatch launches on
 *     its own stream;
 *   FELOG_SERVE_PERSISTENT: jobs with P (K + 2) <= 8192 take the persistent
 *     update; one slot only (slots > 1 is FELOG_EINVAL), so that one
 *     cooperative launch is in flight at a time;
 *   FELOG_SERVE_SHARED: jobs with P (K + 2) <= 8192 train in persistent
 *     launches shared by up to 8 running jobs of equal d: each launch plans
 *     and updates the next 64 minibatches of every job in it, phase by phase
 *     together, on one more stream of the server; other jobs as LAUNCHES.
 * Streams: one per slot, plus one in FELOG_SERVE_SHARED; slots is at most 4
 * (3 in FELOG_SERVE_SHARED, 1 in FELOG_SERVE_PERSISTENT), the device's
 * hardware queues per process. */
enum { FELOG_SERVE_LAUNCHES = 0, FELOG_SERVE_PERSISTENT = 1, FELOG_SERVE_SHARED = 2 };

typedef struct felog_job_desc {
    int32_t n_nodes;
    int64_t nnz;
    const int64_t* indptr;    /* symmetric CSR as for felog_graph_load_csr; copied at  */
    const int32_t* indices;   /* submission                                            */
    int32_t dim;              /* 64, 128 or 256                                        */
    int32_t walks_per_node;   /* r                                                     */
    int32_t walk_length;      /* L                                                     */
    int32_t window;           /* w                                                     */
    uint64_t seed;            /* the job's Philox key (walks, init, negatives)         */
    double arrival_time;      /* scheduled arrival on the server clock (s); 0 = now    */
} felog_job_desc;

enum { FELOG_JOB_QUEUED = 0, FELOG_JOB_RUNNING = 1, FELOG_JOB_DONE = 2, FELOG_JOB_FAILED = 3 };

typedef struct felog_job_state {
    int32_t state;
    double t_arrive, t_admit, t_done;   /* server clock (s); latency = t_done - t_arrive */
    int64_t pairs;
    double loss;
    uint64_t device_bytes;              /* the job's admission estimate (its reservation) */
    int64_t minibatch_pairs;            /* the P the job ran with                          */
    uint64_t peak_bytes;                /* device bytes the job held at its peak; a job   */
                                        /* never holds more than its reservation: an      */
                                        /* allocation beyond it fails the job (ENOMEM)    */
} felog_job_state;

/* A server with `slots` worker threads on `device`.  Jobs queue in arrival order;
 * the head job is admitted when a slot is free and its estimated device bytes
 * fit hbm_budget_bytes minus those of the running jobs (0 = no budget).  The head
 * is never bypassed, so no job starves.  An admitted job runs uniform walks, the
 * degree^0.75 noise table and one training epoch on its own stream; its in-table
 * is then copied to host memory and its device memory released. */
felog_status felog_server_create(int device, uint64_t hbm_budget_bytes,
                                 const felog_server_params* params, felog_server** out);
/* Queue a job (the CSR is copied); a job larger than the whole budget gives EINVAL. */
felog_status felog_server_submit(felog_server* s, const felog_job_desc* job, uint64_t* job_id);
felog_status felog_server_poll(felog_server* s, uint64_t job_id, felog_job_state* state);
/* Block until the job is done or failed (timeout_s < 0: no limit). */
felog_status felog_server_wait(felog_server* s, uint64_t job_id, double timeout_s,
                               felog_job_state* state);
/* Copy a done job's in-table (float32 [n][d]) to host memory. */
felog_status felog_server_fetch(felog_server* s, uint64_t job_id, float* host, int64_t cap);
/* Forget a finished job and its result. */
felog_status felog_server_release(felog_server* s, uint64_t job_id);
/* Server clock (s since creation), peak admitted estimate (bytes), queued jobs. */
felog_status felog_server_stats(felog_server* s, double* clock_s, uint64_t* peak_reserved,
                                int64_t* queued);
/* Finish the running jobs, drop the queued ones, stop the workers. */
void felog_server_destroy(felog_server* s);

#ifdef __cplusplus
}
#endif
#endif /* FELOG_H */
