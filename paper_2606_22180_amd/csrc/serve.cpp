// Serving loop: continuous admission of embedding jobs under an HBM budget.
//
// Each job embeds its own graph with the hot path (uniform walks, one SGNS
// epoch, degree^0.75 noise; no feedback rounds).  Jobs wait in a FIFO queue;
// a job is admitted when one of the worker slots is free and its estimated
// device footprint fits the remaining budget.  The head of the queue is never
// bypassed, so every job is admitted after finitely many earlier jobs finish
// (no starvation).  An admitted job runs on its worker's own HIP stream (one
// stream per job: the id launches of its minibatches go to the same stream),
// so the kernels of the jobs in flight overlap on the GPU's hardware queues;
// its in-table is copied to host memory at the end and its device memory is
// released for the next admission.  Update modes:
//   launches    (default) each job's per-minibatch launches on its stream;
//   persistent  jobs whose minibatches fit the persistent update run it on
//               their own streams with 1 / slots of the compute units each,
//               so the launches of all running jobs can be resident at once
//               and none waits at a grid barrier for workgroups that another
//               job's launch keeps from starting.  Measured on MI355X with
//               four slots, a 219-node job that takes 0.19 s alone finished
//               only with the three larger jobs beside it, after 2.4 s (its
//               launches waited behind theirs);
//   shared      a batcher thread runs the persistent update of up to
//               kMaxBatchJobs running jobs of equal d in shared launches:
//               each plans and updates the next launch group of every job in
//               it, phase by phase together (one grid barrier per phase for
//               all of them).  A job joins at the next launch after its walks
//               and tables are ready and leaves when its minibatches are done.
// A job's results depend only on its own inputs: its RNG counters and
// minibatch sequence are job-local, and every mode gives bit-identical tables.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "common.h"

struct felog_server;

namespace felog {

struct Job {
    uint64_t id = 0;
    felog_job_desc desc{};
    std::vector<int64_t> indptr;
    std::vector<int32_t> indices;
    uint64_t est_bytes = 0;
    uint64_t peak_bytes = 0;
    int64_t minibatch = 0;       // P of this job
    int32_t state = FELOG_JOB_QUEUED;
    double t_arrive = 0, t_admit = 0, t_done = 0;
    int64_t pairs = 0;
    double loss = 0;
    std::string error;
    std::vector<float> result;   // in-table [n][d]
};

struct Server {
    int device = 0;
    uint64_t budget = 0;
    felog_server_params params{};
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_id = 1;
    uint64_t reserved = 0;       // estimated bytes of the running jobs
    uint64_t peak_reserved = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    // shared persistent launches (update_mode FELOG_SERVE_SHARED)
    struct BatchEntry {
        SmallJob* job = nullptr;
        bool done = false;
        std::string err;
        felog_train_stats st{};
    };
    std::thread batcher;
    std::mutex bmu;
    std::condition_variable bcv;
    std::deque<BatchEntry*> bq;          // jobs in training, in arrival order
    bool bstop = false;
    int bblocks = 0;                     // grid of the shared launches

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Minibatch of a job on n nodes: the server's P, capped at the next power of two
// >= n.  Minibatch updates are sums, so with P far above n every row takes
// hundreds of summed steps per minibatch and training diverges.
static int64_t job_minibatch(const felog_job_desc& d, const felog_server_params& p)
{
    int64_t cap = 1;
    while (cap < (int64_t)d.n_nodes) cap <<= 1;
    return std::min<int64_t>(p.minibatch_pairs, cap);
}

// Upper bound of a job's device bytes: every buffer the job allocates, counted
// as if all were held at once (temporaries of the noise build and the walk
// compaction included).
static uint64_t estimate_bytes(const felog_job_desc& d, const felog_server_params& p)
{
    const uint64_t n = (uint64_t)d.n_nodes, nnz = std::max<uint64_t>((uint64_t)d.nnz, 1);
    const uint64_t dim = (uint64_t)d.dim;
    const uint64_t W = n * (uint64_t)d.walks_per_node, L = (uint64_t)d.walk_length;
    const uint64_t P = (uint64_t)job_minibatch(d, p), K = (uint64_t)p.negatives;
    uint64_t pow2 = 1;
    while (pow2 < n) pow2 <<= 1;
    uint64_t b = 0;
    b += 8 * (n + 1) + 4 * nnz + 4 * n + 16;                     // CSR, row maxima, check word
    b += 8 * n * dim + 16 * n + 4 * 16 * kIdSets + 24 + 16;      // tables, counters, offsets
    b += 4 * n + 8 * n + 8 * (n / 2048 + 2) + 8 * (n + 1) + 4 * std::max<uint64_t>(pow2, 2);
    b += 4 * W * L + 4 * W + 4 * (W / 2048 + 2) + 8 * (W / (1u << 20) + 2);   // walks
    const uint64_t T = P * (K + 2);                              // touches per minibatch
    const uint64_t sc = P / 8 + 1 + P * (K + 1) / 8 + 1;         // chunks of split rows
    const uint64_t sr = P / 17 + 1 + P * (K + 1) / 17 + 1;       // split rows
    const uint64_t nbs = P / kScanSpanMin + 1 + P * (K + 1) / kScanSpanMin + 1;  // scan blocks
    b += 16 * n * (kIdSets - 1);                                 // more sets of counters, offsets
    b += kIdSets * (8 * T + 4 * T + 16 * T + 16 * sc + 16 * sr + 24 * nbs);   // id/sort sets
    b += 8 * P * (K + 1) + 4 * T + 4 * P * dim + 8 * sc * dim;   // outputs, keys, split sums
    b += 8 * (P + 4) + 4 * L * 2 * (uint64_t)d.window;           // loss slots, slices
    b += 64 * 16;                                                // small allocations of 16 B
    if (p.update_mode != FELOG_SERVE_LAUNCHES && P * (K + 2) <= (uint64_t)kSmallMaxTouches) {
        // persistent update: plans, per-pair rows, descriptors (B minibatches
        // at most W (L - 1) 2 w / P + one per walk chunk), control words
        const uint64_t B = W * L * 2 * (uint64_t)d.window / P + W / (1u << 20) + 2;
        b += small_path_bytes((int64_t)P, (int)K, (int)dim, (int64_t)B, 256) +
             4 * L * 2 * (uint64_t)d.window;                       // its slices
    }
    return b + b / 16;                                           // headroom
}

static void run_job(Server& s, Job& job)
{
    Ctx ctx;
    ctx.device = s.device;
    ctx.budget = job.est_bytes;   // the job's allocations stay within its reservation
    ctx.make_current();
    FELOG_HIP(hipStreamCreateWithFlags(&ctx.stream, hipStreamNonBlocking));
    hipDeviceProp_t prop;
    FELOG_HIP(hipGetDeviceProperties(&prop, s.device));
    ctx.num_cus = prop.multiProcessorCount;
    // One stream per job.  The persistent mode has one slot, so the job's
    // cooperative launch is the only one in flight; it takes the default
    // grid (64 workgroups).
    ctx.single_stream = true;
    ctx.sgns_path = s.params.update_mode == FELOG_SERVE_PERSISTENT ? 0 : 1;
    ctx.sgns_blocks = std::max(1, std::min(64, ctx.num_cus / std::max(1, s.params.slots)));
    FELOG_HIP(hipEventCreate(&ctx.ev0));
    FELOG_HIP(hipEventCreate(&ctx.ev1));
    struct StreamGuard {
        Ctx& c;
        ~StreamGuard()
        {
            (void)hipStreamSynchronize(c.stream);
            c.release_aux();
            (void)hipEventDestroy(c.ev0);
            (void)hipEventDestroy(c.ev1);
            (void)hipStreamDestroy(c.stream);
        }
    } guard{ctx};
    {
        const felog_job_desc& d = job.desc;
        Graph g;
        g.ctx = &ctx;
        g.n = d.n_nodes;
        g.nnz = d.nnz;
        g.indptr.alloc(&ctx, sizeof(int64_t) * (g.n + 1));
        g.indices.alloc(&ctx, sizeof(int32_t) * std::max<int64_t>(g.nnz, 1));
        FELOG_HIP(hipMemcpyAsync(g.indptr.ptr, job.indptr.data(), sizeof(int64_t) * (g.n + 1),
                                 hipMemcpyHostToDevice, ctx.stream));
        if (g.nnz)
            FELOG_HIP(hipMemcpyAsync(g.indices.ptr, job.indices.data(), sizeof(int32_t) * g.nnz,
                                     hipMemcpyHostToDevice, ctx.stream));
        DevBuf bad;
        bad.alloc(&ctx, sizeof(unsigned long long));
        launch_validate_graph(g, bad.as<unsigned long long>());
        unsigned long long code = 0;
        FELOG_HIP(hipMemcpyAsync(&code, bad.ptr, sizeof code, hipMemcpyDeviceToHost, ctx.stream));
        ctx.sync();
        FELOG_REQUIRE(code == ~0ull, "job graph is not a valid symmetric CSR (row %llu)",
                      (unsigned long long)(code >> 3));
        launch_row_wmax(g);

        Model m;
        m.ctx = &ctx;
        m.g = &g;
        m.dim = d.dim;
        m.neg_dist = FELOG_NEG_DEGREE;
        const size_t tb = sizeof(float) * (size_t)g.n * d.dim;
        m.tin.alloc(&ctx, tb);
        m.tout.alloc(&ctx, tb);
        model_alloc_update_state(m);
        launch_init_tables(m, d.seed);
        {
            DevBuf counts;
            counts.alloc(&ctx, sizeof(uint32_t) * g.n);
            launch_degree_counts(g, counts.as<uint32_t>());
            build_noise_from_counts(m, counts.as<uint32_t>());
        }
        Walks w;
        w.g = &g;
        w.L = d.walk_length;
        w.W = (int64_t)g.n * d.walks_per_node;
        w.id_base = 0;
        w.data.alloc(&ctx, sizeof(int32_t) * std::max<int64_t>(w.W * w.L, 1));
        felog_walk_params wp{};
        wp.kind = FELOG_WALK_UNIFORM;
        wp.walks_per_node = d.walks_per_node;
        wp.length = d.walk_length;
        wp.seed = d.seed;
        wp.id_base = 0;
        launch_walks(w, wp, nullptr, g.n);
        felog_train_params tp{};
        tp.window = d.window;
        tp.negatives = s.params.negatives;
        tp.lr_start = s.params.lr_start;
        tp.lr_end = s.params.lr_end;
        tp.minibatch_pairs = job.minibatch;
        tp.chunk_walks = 0;
        tp.seed = d.seed;
        felog_train_stats st{};
        if (s.params.update_mode == FELOG_SERVE_SHARED && small_job_fits(m, tp)) {
            // training in the batcher's shared launches
            SmallJobPtr sj = small_job_begin(m, w, tp, s.bblocks);
            Server::BatchEntry e;
            e.job = sj.get();
            {
                std::unique_lock<std::mutex> lk(s.bmu);
                s.bq.push_back(&e);
                s.bcv.notify_all();
                s.bcv.wait(lk, [&] { return e.done; });
            }
            FELOG_REQUIRE(e.err.empty(), "%s", e.err.c_str());
            st = e.st;
        } else {
            train_minibatches(m, w, tp, 0, -1, true, &st, nullptr, nullptr, 0, nullptr, nullptr,
                              nullptr, 0, nullptr);
        }
        job.result.resize((size_t)g.n * d.dim);
        FELOG_HIP(hipMemcpyAsync(job.result.data(), m.tin.ptr, tb, hipMemcpyDeviceToHost,
                                 ctx.stream));
        ctx.sync();
        job.pairs = st.pairs;
        job.loss = st.loss;
        job.peak_bytes = ctx.peak;
    }
}

// The shared launches: each round takes the jobs in training whose d and K
// equal those of the oldest one (up to kMaxBatchJobs), launches their next
// launch group together, waits for it, and hands finished jobs back to their
// workers.  A launch that aborts (a barrier wait exceeded its bound) fails its
// jobs; the barrier words are then reset.
static void batcher_loop(Server* s)
{
    Ctx c;
    c.device = s->device;
    c.make_current();
    hipDeviceProp_t prop;
    std::string setup_err;
    SmallBatchCtl ctl;
    try {
        FELOG_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
        FELOG_HIP(hipGetDeviceProperties(&prop, s->device));
        c.num_cus = prop.multiProcessorCount;
        small_batch_init(ctl, c, s->bblocks);
    } catch (const Error&) {
        setup_err = felog_last_error();
        if (setup_err.empty()) setup_err = "shared launches could not start";
    }
    for (;;) {
        std::vector<Server::BatchEntry*> batch;
        {
            std::unique_lock<std::mutex> lk(s->bmu);
            s->bcv.wait(lk, [&] { return s->bstop || !s->bq.empty(); });
            if (s->bq.empty()) break;   // stopping and nothing in training
            const SmallJob& head = *s->bq.front()->job;
            for (Server::BatchEntry* e : s->bq)
                if ((int)batch.size() < kMaxBatchJobs && small_job_dim(*e->job) == small_job_dim(head) &&
                    small_job_negatives(*e->job) == small_job_negatives(head))
                    batch.push_back(e);
        }
        std::string err = setup_err;
        std::vector<bool> finished(batch.size(), false);
        if (err.empty()) {
            try {
                std::vector<SmallJob*> jobs;
                for (Server::BatchEntry* e : batch) jobs.push_back(e->job);
                small_jobs_step(jobs, ctl, c.stream);
                if (small_batch_aborted(ctl, c.stream)) {
                    err = "shared persistent update: a grid barrier wait exceeded its bound";
                    small_batch_init(ctl, c, s->bblocks);
                } else {
                    for (size_t i = 0; i < batch.size(); ++i)
                        if (small_job_done(*batch[i]->job)) {
                            small_job_end(*batch[i]->job, c.stream, &batch[i]->st);
                            finished[i] = true;
                        }
                }
            } catch (const Error&) {
                err = felog_last_error();
                if (err.empty()) err = "shared persistent update failed";
            } catch (...) {
                err = "shared persistent update failed with an unexpected internal error";
            }
        }
        {
            std::lock_guard<std::mutex> lk(s->bmu);
            for (size_t i = 0; i < batch.size(); ++i) {
                if (!err.empty()) batch[i]->err = err;
                if (!err.empty() || finished[i]) {
                    batch[i]->done = true;
                    s->bq.erase(std::find(s->bq.begin(), s->bq.end(), batch[i]));
                }
            }
        }
        s->bcv.notify_all();
    }
    if (c.stream) {
        (void)hipStreamSynchronize(c.stream);
        ctl.words.release();
        (void)hipStreamDestroy(c.stream);
    }
}

static void worker_loop(Server* s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        std::shared_ptr<Job> job;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] {
                if (s->stopping) return true;
                if (s->queue.empty()) return false;
                const Job& head = *s->jobs[s->queue.front()];
                return s->budget == 0 || s->reserved + head.est_bytes <= s->budget;
            });
            if (s->stopping) return;
            job = s->jobs[s->queue.front()];
            s->queue.pop_front();
            s->reserved += job->est_bytes;
            s->peak_reserved = std::max(s->peak_reserved, s->reserved);
            job->state = FELOG_JOB_RUNNING;
            job->t_admit = s->now();
        }
        std::string err;
        try {
            run_job(*s, *job);
        } catch (const Error&) {
            err = felog_last_error();
            if (err.empty()) err = "job failed";
        } catch (...) {
            err = "job failed with an unexpected internal error";
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->reserved -= job->est_bytes;
            job->t_done = s->now();
            job->state = err.empty() ? FELOG_JOB_DONE : FELOG_JOB_FAILED;
            job->error = err;
            job->indptr.clear();
            job->indptr.shrink_to_fit();
            job->indices.clear();
            job->indices.shrink_to_fit();
        }
        s->cv.notify_all();
    }
}

}  // namespace felog

using namespace felog;

struct felog_server : Server {};

template <class F>
static felog_status guarded_s(F&& body)
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

#define NEED_S(p) FELOG_REQUIRE((p) != nullptr, "%s must not be NULL", #p)

extern "C" {

felog_status felog_server_create(int device, uint64_t hbm_budget_bytes,
                                 const felog_server_params* params, felog_server** out)
{
    return guarded_s([&] {
        NEED_S(params);
        NEED_S(out);
        *out = nullptr;
        int n = 0;
        FELOG_HIP(hipGetDeviceCount(&n));
        FELOG_REQUIRE(device >= 0 && device < n, "device %d out of range", device);
        FELOG_REQUIRE(params->update_mode == FELOG_SERVE_LAUNCHES ||
                          params->update_mode == FELOG_SERVE_PERSISTENT ||
                          params->update_mode == FELOG_SERVE_SHARED,
                      "unknown update_mode %d", params->update_mode);
        // The persistent mode runs one job at a time: with several slots, the
        // jobs' cooperative launches would be in flight together on separate
        // streams, and whether they are all resident at once is up to the
        // runtime and the dispatcher, not to this library (the shared mode
        // puts the jobs into one cooperative launch instead).
        const int max_slots = params->update_mode == FELOG_SERVE_SHARED       ? 3
                              : params->update_mode == FELOG_SERVE_PERSISTENT ? 1
                                                                              : 4;
        FELOG_REQUIRE(params->slots >= 1 && params->slots <= max_slots,
                      "slots must be in [1, %d] (%s; the device has 4 hardware queues per "
                      "process)", max_slots,
                      params->update_mode == FELOG_SERVE_SHARED
                          ? "one stream each, plus the shared launches'"
                          : params->update_mode == FELOG_SERVE_PERSISTENT
                                ? "one cooperative launch in flight at a time"
                                : "one stream each");
        FELOG_REQUIRE(params->minibatch_pairs >= 1 && params->minibatch_pairs <= (1 << 24),
                      "minibatch_pairs must be in [1, 2^24]");
        FELOG_REQUIRE(params->negatives >= 1 && params->negatives <= 20,
                      "negatives must be in [1, 20]");
        auto s = std::make_unique<felog_server>();
        s->device = device;
        s->budget = hbm_budget_bytes;
        s->params = *params;
        s->t0 = std::chrono::steady_clock::now();
        if (params->update_mode == FELOG_SERVE_SHARED) {
            // one grid for every shared launch: resident for each d
            Ctx probe;
            probe.device = device;
            hipDeviceProp_t prop;
            FELOG_HIP(hipGetDeviceProperties(&prop, device));
            probe.num_cus = prop.multiProcessorCount;
            int blocks = 1 << 30;
            for (int d : {64, 128, 256})
                blocks = std::min(blocks, small_update_blocks(probe, d, params->negatives));
            s->bblocks = blocks;
            s->batcher = std::thread(batcher_loop, s.get());
        }
        for (int i = 0; i < params->slots; ++i) s->workers.emplace_back(worker_loop, s.get());
        *out = s.release();
    });
}

felog_status felog_server_submit(felog_server* s, const felog_job_desc* d, uint64_t* job_id)
{
    return guarded_s([&] {
        NEED_S(s);
        NEED_S(d);
        NEED_S(job_id);
        FELOG_REQUIRE(d->n_nodes >= 1 && d->nnz >= 0 && d->indptr, "bad job graph");
        FELOG_REQUIRE(d->nnz == 0 || d->indices, "indices must not be NULL when nnz > 0");
        FELOG_REQUIRE(d->dim == 64 || d->dim == 128 || d->dim == 256, "dim must be 64/128/256");
        FELOG_REQUIRE(d->walks_per_node >= 1 && d->walk_length >= 1 && d->walk_length <= 65536,
                      "bad walk parameters");
        FELOG_REQUIRE(d->window >= 1 && d->window <= 127, "window must be in [1, 127]");
        FELOG_REQUIRE(d->indptr[0] == 0 && d->indptr[d->n_nodes] == d->nnz,
                      "indptr must start at 0 and end at nnz");
        auto job = std::make_shared<Job>();
        job->desc = *d;
        job->indptr.assign(d->indptr, d->indptr + d->n_nodes + 1);
        job->indices.assign(d->indices, d->indices + d->nnz);
        job->desc.indptr = nullptr;
        job->desc.indices = nullptr;
        job->est_bytes = estimate_bytes(*d, s->params);
        job->minibatch = job_minibatch(*d, s->params);
        FELOG_REQUIRE(s->budget == 0 || job->est_bytes <= s->budget,
                      "job needs about %llu device bytes, more than the server's budget %llu",
                      (unsigned long long)job->est_bytes, (unsigned long long)s->budget);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            job->id = s->next_id++;
            job->t_arrive = d->arrival_time > 0 ? d->arrival_time : s->now();
            s->jobs[job->id] = job;
            s->queue.push_back(job->id);
            *job_id = job->id;
        }
        s->cv.notify_all();
    });
}

static void fill_state(const Job& j, felog_job_state* st)
{
    st->state = j.state;
    st->t_arrive = j.t_arrive;
    st->t_admit = j.t_admit;
    st->t_done = j.t_done;
    st->pairs = j.pairs;
    st->loss = j.loss;
    st->device_bytes = j.est_bytes;
    st->peak_bytes = j.peak_bytes;
    st->minibatch_pairs = j.minibatch;
}

felog_status felog_server_poll(felog_server* s, uint64_t job_id, felog_job_state* st)
{
    return guarded_s([&] {
        NEED_S(s);
        NEED_S(st);
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(job_id);
        FELOG_REQUIRE(it != s->jobs.end(), "unknown job %llu", (unsigned long long)job_id);
        fill_state(*it->second, st);
    });
}

felog_status felog_server_wait(felog_server* s, uint64_t job_id, double timeout_s,
                               felog_job_state* st)
{
    return guarded_s([&] {
        NEED_S(s);
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->jobs.find(job_id);
        FELOG_REQUIRE(it != s->jobs.end(), "unknown job %llu", (unsigned long long)job_id);
        std::shared_ptr<Job> j = it->second;
        auto done = [&] { return j->state == FELOG_JOB_DONE || j->state == FELOG_JOB_FAILED; };
        if (timeout_s < 0) s->cv.wait(lk, done);
        else s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
        if (st) fill_state(*j, st);
        FELOG_REQUIRE(done(), "job %llu not finished within the timeout",
                      (unsigned long long)job_id);
        if (j->state == FELOG_JOB_FAILED) fail(FELOG_EDEVICE, "job %llu failed: %s",
                                               (unsigned long long)job_id, j->error.c_str());
    });
}

felog_status felog_server_fetch(felog_server* s, uint64_t job_id, float* host, int64_t cap)
{
    return guarded_s([&] {
        NEED_S(s);
        NEED_S(host);
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(job_id);
        FELOG_REQUIRE(it != s->jobs.end(), "unknown job %llu", (unsigned long long)job_id);
        Job& j = *it->second;
        if (j.state != FELOG_JOB_DONE)
            fail(FELOG_ESTATE, "job %llu is not done", (unsigned long long)job_id);
        FELOG_REQUIRE(cap >= (int64_t)j.result.size(), "buffer holds %lld floats, need %lld",
                      (long long)cap, (long long)j.result.size());
        std::memcpy(host, j.result.data(), sizeof(float) * j.result.size());
    });
}

felog_status felog_server_release(felog_server* s, uint64_t job_id)
{
    return guarded_s([&] {
        NEED_S(s);
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(job_id);
        FELOG_REQUIRE(it != s->jobs.end(), "unknown job %llu", (unsigned long long)job_id);
        if (it->second->state == FELOG_JOB_QUEUED || it->second->state == FELOG_JOB_RUNNING)
            fail(FELOG_ESTATE, "job %llu has not finished", (unsigned long long)job_id);
        s->jobs.erase(it);
    });
}

felog_status felog_server_stats(felog_server* s, double* clock_s, uint64_t* peak_reserved,
                                int64_t* queued)
{
    return guarded_s([&] {
        NEED_S(s);
        std::lock_guard<std::mutex> lk(s->mu);
        if (clock_s) *clock_s = s->now();
        if (peak_reserved) *peak_reserved = s->peak_reserved;
        if (queued) *queued = (int64_t)s->queue.size();
    });
}

void felog_server_destroy(felog_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_all();
    for (auto& t : s->workers) t.join();   // running jobs finish (with the batcher's help)
    if (s->batcher.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->bmu);
            s->bstop = true;
        }
        s->bcv.notify_all();
        s->batcher.join();
    }
    delete s;
}

}  // extern "C"
