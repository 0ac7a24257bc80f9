// Serving: continuous batching of independent spin systems (see the
// serving section of include/sllg.h).
//
// Each request becomes one replica of a Batch whose buffers come from a
// pooled allocation of the HBM budget.  A scheduler thread loops: admit
// queued requests in arrival order while slots and budget allow, advance
// every active replica by up to one chunk of steps with one batched launch
// sequence (a replayed HIP graph), then retire finished or cancelled
// replicas and free their memory for the queue.  A request that arrives
// while others run starts at the next chunk boundary.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sllg.h"
#include "batch.hpp"
#include "prepare.hpp"

using namespace sllg;

namespace {

constexpr int kAvgBlocks = 10;

struct Job {
    uint64_t ticket = 0;
    HostStructure st;
    HostMaterials mat;
    Dynamics dyn;
    std::vector<double> S0;
    int64_t n = 0, n_steps = 0, n_avg = 0;
    bool record = false;
    size_t bytes = 0;
    // progress
    int state = SLLG_REQ_QUEUED;
    int status = SLLG_OK;
    int slot = -1;
    int64_t steps_done = 0;
    bool cancel = false;
    double t_submit = 0, t_start = 0, t_done = 0;
    // results
    std::vector<double> S_final, m_series, E_series;
    double m[3] = {0, 0, 0}, E = 0, avg[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

struct ServerBase {
    virtual ~ServerBase() = default;
    virtual int admit(Job& j) = 0;                          // returns slot
    virtual void prepare_chunk(Job& j, int K) = 0;           // nsteps, flags
    virtual void run_chunk(int K, hipStream_t st) = 0;
    virtual void harvest(Job& j, hipStream_t st, bool finished) = 0;
    virtual void retire(Job& j) = 0;
    virtual size_t in_use() = 0;
    virtual void set_launch(int remap, int order) = 0;   // launch shape of the next chunks
    virtual int64_t graph_captures() = 0;
};

template <typename R>
struct ServerT final : ServerBase {
    ServerT(int device, size_t budget, int max_active)
        : pool(budget), batch(device, &pool, max_active)
    {
        batch.set_round_grid(true);
    }
    PoolAllocator pool;
    Batch<R> batch;

    int admit(Job& j) override
    {
        const int64_t rec_cap = j.record ? j.n_steps : 1;
        return batch.add(j.st, j.mat, j.dyn, j.S0, std::max<int64_t>(rec_cap, chunk_cap), kAvgBlocks);
    }
    void prepare_chunk(Job& j, int K) override
    {
        ReplicaDev<R>& r = batch.mirror(j.slot);
        const int64_t left = j.n_steps - j.steps_done;
        const int32_t ns = (int32_t)std::min<int64_t>(K, left);
        // keep the structural bits (materials, axes, neighbour layout); set
        // only the per-run ones
        int32_t flags = (r.flags & ~(kRecord | kRecordSeries | kAverage)) | kRecord;
        if (j.record)
            flags |= kRecordSeries;
        if (j.n_avg > 0)
            flags |= kAverage;
        if (r.nsteps != ns || r.flags != flags) {
            r.nsteps = ns;
            r.flags = flags;
            batch.mark_dirty();
        }
        if (j.steps_done == 0 && j.n_avg > 0) {
            const int blocks = (int)std::min<int64_t>(kAvgBlocks, j.n_avg);
            r.avg_blocks = blocks;
            r.avg_block_len = j.n_avg / blocks;
            r.avg_first = (int64_t)j.dyn.step + (j.n_steps - j.n_avg);
            batch.quiesce();
            hip_check(hipMemset(r.acc, 0, sizeof(double) * 5 * kAvgBlocks), "clear sums");
            batch.mark_dirty();
        }
    }
    void run_chunk(int K, hipStream_t st) override { batch.run_chunk(K, st, true); }
    void set_launch(int remap, int order) override
    {
        batch.set_remap(remap);
        batch.set_tile_order(order, 0);
    }
    int64_t graph_captures() override { return batch.graph_captures(); }
    void harvest(Job& j, hipStream_t st, bool finished) override
    {
        (void)st;
        if (!finished)
            return;
        ReplicaDev<R>& r = batch.mirror(j.slot);
        // the last record is the final state: slot rec_pos - 1 with a series,
        // else nsteps - 1 of the last chunk
        const int64_t last = (r.flags & kRecordSeries) ? r.rec_pos - 1 : r.nsteps - 1;
        double rec[4];
        batch.quiesce();
        hip_check(hipMemcpy(rec, r.records + 4 * last, sizeof(rec), hipMemcpyDeviceToHost), "download record");
        j.m[0] = rec[0];
        j.m[1] = rec[1];
        j.m[2] = rec[2];
        j.E = rec[3];
        j.S_final.resize(3 * (size_t)j.n);
        batch.get_spins(j.slot, j.S_final.data(), st);
        if (j.record) {
            std::vector<double> all(4 * (size_t)j.n_steps);
            hip_check(hipMemcpy(all.data(), r.records, all.size() * sizeof(double), hipMemcpyDeviceToHost),
                      "download series");
            j.m_series.resize(3 * (size_t)j.n_steps);
            j.E_series.resize((size_t)j.n_steps);
            for (int64_t t = 0; t < j.n_steps; ++t) {
                j.m_series[3 * t] = all[4 * t];
                j.m_series[3 * t + 1] = all[4 * t + 1];
                j.m_series[3 * t + 2] = all[4 * t + 2];
                j.E_series[t] = all[4 * t + 3];
            }
        }
        if (j.n_avg > 0) {
            double acc[5 * kAvgBlocks];
            hip_check(hipMemcpy(acc, r.acc, sizeof(acc), hipMemcpyDeviceToHost), "download sums");
            averages_from_block_sums(acc, r.avg_blocks, r.avg_block_len, j.avg);
        }
    }
    void retire(Job& j) override
    {
        batch.remove(j.slot);
        j.slot = -1;
    }
    size_t in_use() override { return pool.in_use(); }
    int64_t chunk_cap = 1;
};

}  // namespace

struct sllg_server {
    int device = 0;
    sllg_server_opts opts{};
    std::string err;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    std::vector<uint64_t> active;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    std::unique_ptr<ServerBase> impl;
    hipStream_t stream = nullptr;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    sllg_server_stats stats{};
    std::string fatal;
    // Launch-shape tuning per batch composition (kept for the server's life).
    struct Tuning {
        int next = 0;          // candidate timed next
        int best = 0;
        double best_time = 1e300;   // seconds per spin-step
        bool done = false;
    };
    std::map<uint64_t, Tuning> tuning;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Launch shapes the server tries for each batch composition: XCD mapping
// of the tile ranges and tile order (the grid is always the resident one,
// the tile the largest).  Results do not depend on them.
struct LaunchShape {
    int remap, order;
};
constexpr LaunchShape kServerShapes[] = {{1, 1}, {1, 0}, {0, 1}, {0, 0}, {2, 1}, {2, 0}};
constexpr int kNumServerShapes = (int)(sizeof(kServerShapes) / sizeof(kServerShapes[0]));

int ceil_log2(double x)
{
    int k = 0;
    while (k < 62 && (double)(int64_t(1) << k) < x)
        ++k;
    return k;
}

// A batch composition, bucketed: the number of requests that run and their
// total spins, each to the next power of two.
uint64_t composition_key(const std::vector<Job*>& run)
{
    double sites = 0.0;
    for (const Job* j : run)
        sites += (double)j->n;
    return ((uint64_t)ceil_log2((double)run.size()) << 8) | (uint64_t)ceil_log2(sites);
}

void finish(sllg_server* s, Job& j, int state, int status)
{
    j.state = state;
    j.status = status;
    j.t_done = s->now();
    if (state == SLLG_REQ_DONE)
        s->stats.completed++;
    else if (state == SLLG_REQ_FAILED)
        s->stats.failed++;
    else if (state == SLLG_REQ_CANCELLED)
        s->stats.cancelled++;
}

void scheduler(sllg_server* s)
{
    (void)hipSetDevice(s->device);
    const int K = s->opts.chunk_steps;
    for (;;) {
        std::vector<Job*> run;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->active.empty(); });
            if (s->stop)
                break;
            // retire cancelled active jobs
            for (auto it = s->active.begin(); it != s->active.end();) {
                Job& j = *s->jobs[*it];
                if (j.cancel) {
                    try {
                        s->impl->retire(j);
                    } catch (const Failure&) {
                    }
                    finish(s, j, SLLG_REQ_CANCELLED, SLLG_E_CANCELLED);
                    it = s->active.erase(it);
                    s->done_cv.notify_all();
                } else {
                    ++it;
                }
            }
            // admit in arrival order while memory and slots allow
            while (!s->queue.empty() && (int)s->active.size() < s->opts.max_active) {
                Job& j = *s->jobs[s->queue.front()];
                if (j.cancel) {
                    finish(s, j, SLLG_REQ_CANCELLED, SLLG_E_CANCELLED);
                    s->queue.pop_front();
                    s->done_cv.notify_all();
                    continue;
                }
                if (s->impl->in_use() + j.bytes > s->opts.hbm_budget)
                    break;
                try {
                    j.slot = s->impl->admit(j);
                } catch (const Failure& f) {
                    if (f.code == SLLG_E_BUDGET && !s->active.empty())
                        break;   // fragmented: wait for memory to free up
                    finish(s, j, SLLG_REQ_FAILED, f.code);
                    s->queue.pop_front();
                    s->done_cv.notify_all();
                    continue;
                }
                j.state = SLLG_REQ_RUNNING;
                j.t_start = s->now();
                s->active.push_back(j.ticket);
                s->queue.pop_front();
            }
            for (uint64_t t : s->active)
                run.push_back(s->jobs[t].get());
            s->stats.active = (int64_t)s->active.size();
            s->stats.queued = (int64_t)s->queue.size();
            s->stats.hbm_in_use = s->impl->in_use();
        }
        if (run.empty())
            continue;
        // one chunk for every active replica; the lock is not held while the
        // GPU works, so clients can submit, poll and cancel meanwhile.  A new
        // batch composition times each launch shape on its chunks (a chunk
        // that captured a graph does not count) and then keeps the fastest.
        sllg_server::Tuning& tune = s->tuning[composition_key(run)];
        const int shape = tune.done ? tune.best : tune.next;
        const double t_begin = s->now();
        double spin_steps = 0.0;
        bool captured = false;
        try {
            s->impl->set_launch(kServerShapes[shape].remap, kServerShapes[shape].order);
            for (Job* j : run) {
                s->impl->prepare_chunk(*j, K);
                spin_steps += (double)j->n * (double)std::min<int64_t>(K, j->n_steps - j->steps_done);
            }
            const int64_t captures = s->impl->graph_captures();
            s->impl->run_chunk(K, s->stream);
            hip_check(hipStreamSynchronize(s->stream), "chunk");
            captured = s->impl->graph_captures() != captures;
        } catch (const Failure& f) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->fatal = f.msg;
            for (Job* j : run) {
                try {
                    s->impl->retire(*j);
                } catch (const Failure&) {
                }
                finish(s, *j, SLLG_REQ_FAILED, f.code);
            }
            s->active.clear();
            s->done_cv.notify_all();
            continue;
        }
        const double t_chunk = s->now() - t_begin;
        bool newly_tuned = false;
        if (!tune.done && !captured && spin_steps > 0.0) {
            const double per = t_chunk / spin_steps;
            if (per < tune.best_time) {
                tune.best_time = per;
                tune.best = shape;
            }
            if (++tune.next == kNumServerShapes)
                tune.done = newly_tuned = true;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.chunks++;
        s->stats.spin_steps += spin_steps;
        s->stats.busy_seconds += t_chunk;
        if (newly_tuned)
            s->stats.tuned_compositions++;
        s->stats.last_xcd_remap = kServerShapes[shape].remap;
        s->stats.last_tile_order = kServerShapes[shape].order;
        for (auto it = s->active.begin(); it != s->active.end();) {
            Job& j = *s->jobs[*it];
            j.steps_done += std::min<int64_t>(K, j.n_steps - j.steps_done);
            const bool finished = j.steps_done >= j.n_steps;
            if (finished) {
                int state = SLLG_REQ_DONE, status = SLLG_OK;
                try {
                    s->impl->harvest(j, s->stream, true);
                    if (!std::isfinite(j.E)) {
                        state = SLLG_REQ_FAILED;
                        status = SLLG_E_NUMERIC;
                    }
                    s->impl->retire(j);
                } catch (const Failure& f) {
                    state = SLLG_REQ_FAILED;
                    status = f.code;
                }
                finish(s, j, state, status);
                it = s->active.erase(it);
                s->done_cv.notify_all();
            } else {
                ++it;
            }
        }
        s->stats.hbm_in_use = s->impl->in_use();
    }
}

}  // namespace

extern "C" {

sllg_status sllg_server_create(int device, const sllg_server_opts* opts, sllg_server** out)
{
    if (!out || !opts)
        return SLLG_E_ARG;
    *out = nullptr;
    if (opts->hbm_budget < (size_t(1) << 20) || opts->max_active < 1 || opts->max_active > 4096 ||
        opts->chunk_steps < 2 || opts->chunk_steps > 4096 || (opts->chunk_steps & 1) ||
        (opts->precision != SLLG_FP32 && opts->precision != SLLG_FP64))
        return SLLG_E_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return SLLG_E_DEVICE;
    auto s = std::make_unique<sllg_server>();
    s->device = device;
    s->opts = *opts;
    try {
        hip_check(hipSetDevice(device), "hipSetDevice");
        hip_check(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
        if (opts->precision == SLLG_FP32) {
            auto* impl = new ServerT<float>(device, opts->hbm_budget, opts->max_active);
            impl->chunk_cap = opts->chunk_steps;
            s->impl.reset(impl);
        } else {
            auto* impl = new ServerT<double>(device, opts->hbm_budget, opts->max_active);
            impl->chunk_cap = opts->chunk_steps;
            s->impl.reset(impl);
        }
    } catch (const Failure& f) {
        if (s->stream)
            (void)hipStreamDestroy(s->stream);
        return f.code;
    }
    s->stats.hbm_budget = opts->hbm_budget;
    sllg_server* raw = s.release();
    raw->worker = std::thread(scheduler, raw);
    *out = raw;
    return SLLG_OK;
}

void sllg_server_destroy(sllg_server* srv)
{
    if (!srv)
        return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->worker.joinable())
        srv->worker.join();
    (void)hipSetDevice(srv->device);
    for (uint64_t t : srv->active) {
        try {
            srv->impl->retire(*srv->jobs[t]);
        } catch (const Failure&) {
        }
    }
    srv->impl.reset();
    if (srv->stream)
        (void)hipStreamDestroy(srv->stream);
    delete srv;
}

const char* sllg_server_last_error(const sllg_server* srv) { return srv ? srv->err.c_str() : ""; }

double sllg_server_clock(const sllg_server* srv) { return srv ? srv->now() : 0.0; }

sllg_status sllg_submit(sllg_server* srv, const sllg_request* req, uint64_t* ticket)
{
    if (!srv || !req || !ticket)
        return SLLG_E_ARG;
    auto j = std::make_unique<Job>();
    try {
        if (req->n_spins < 1 || req->n_spins >= (int64_t(1) << kColBits))
            fail(SLLG_E_ARG, "n_spins must be in 1 .. 2^28-1");
        if (req->n_steps < 1)
            fail(SLLG_E_ARG, "n_steps must be >= 1");
        if (req->n_avg < 0 || req->n_avg > req->n_steps)
            fail(SLLG_E_ARG, "n_avg must be in 0 .. n_steps");
        j->n = req->n_spins;
        j->st = build_structure(req->n_spins, req->row_ptr, req->col, req->ntype, req->J, req->n_types, true,
                                kHaloCap);
        // a batch has parallelism across requests: the largest tiles keep
        // the per-tile overheads lowest
        j->st.tile_request = -1;
        j->mat = build_materials(req->n_spins, req->mu_s, req->k_u, req->easy_axis, req->per_site);
        j->dyn.alpha = req->alpha;
        j->dyn.gamma = req->gamma;
        j->dyn.dt = req->dt;
        j->dyn.temperature = req->temperature;
        for (int c = 0; c < 3; ++c)
            j->dyn.H[c] = req->H_app[c];
        j->dyn.seed = req->seed;
        j->dyn.step = 0;
        check_dynamics(j->dyn);
        if (req->S0) {
            j->S0 = normalised_spins(req->n_spins, req->S0);
        } else {
            j->S0.assign(3 * (size_t)req->n_spins, 0.0);
            for (int64_t i = 0; i < req->n_spins; ++i)
                j->S0[3 * i + 2] = 1.0;
        }
        j->n_steps = req->n_steps;
        j->n_avg = req->n_avg;
        j->record = req->record != 0;
        const int64_t rec_cap = std::max<int64_t>(j->record ? j->n_steps : 1, srv->opts.chunk_steps);
        j->bytes = replica_bytes(j->st, j->mat, srv->opts.precision == SLLG_FP32 ? 4 : 8, rec_cap, kAvgBlocks);
        if (j->bytes > srv->opts.hbm_budget)
            fail(SLLG_E_BUDGET, "request needs " + std::to_string(j->bytes) + " bytes, more than the budget");
    } catch (const Failure& f) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->err = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->err = "host allocation failed";
        return SLLG_E_NOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        j->ticket = srv->next_ticket++;
        j->t_submit = srv->now();
        *ticket = j->ticket;
        srv->queue.push_back(j->ticket);
        srv->jobs[j->ticket] = std::move(j);
        srv->stats.submitted++;
        srv->err.clear();
    }
    srv->cv.notify_all();
    return SLLG_OK;
}

namespace {
void fill_result(const Job& j, sllg_result* r)
{
    r->state = j.state;
    r->status = j.status;
    r->n_spins = j.n;
    r->n_steps = j.n_steps;
    r->steps_done = j.steps_done;
    for (int c = 0; c < 3; ++c)
        r->m[c] = j.m[c];
    r->E = j.E;
    for (int c = 0; c < 8; ++c)
        r->avg[c] = j.avg[c];
    r->t_submit = j.t_submit;
    r->t_start = j.t_start;
    r->t_done = j.t_done;
    r->hbm_bytes = j.bytes;
}
bool settled(int state) { return state >= SLLG_REQ_DONE; }
}  // namespace

sllg_status sllg_poll(sllg_server* srv, uint64_t ticket, sllg_result* result)
{
    if (!srv || !result)
        return SLLG_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end())
        return SLLG_E_ARG;
    fill_result(*it->second, result);
    return SLLG_OK;
}

sllg_status sllg_wait(sllg_server* srv, uint64_t ticket, double timeout_s, sllg_result* result)
{
    if (!srv)
        return SLLG_E_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end())
        return SLLG_E_ARG;
    Job* j = it->second.get();
    const bool ok = srv->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                          [&] { return settled(j->state); });
    if (result)
        fill_result(*j, result);
    return ok ? SLLG_OK : SLLG_E_STATE;
}

sllg_status sllg_fetch(sllg_server* srv, uint64_t ticket, double* S_out, double* m_series, double* E_series)
{
    if (!srv)
        return SLLG_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end())
        return SLLG_E_ARG;
    const Job& j = *it->second;
    if (j.state != SLLG_REQ_DONE)
        return SLLG_E_STATE;
    if (S_out)
        std::memcpy(S_out, j.S_final.data(), j.S_final.size() * sizeof(double));
    if ((m_series || E_series) && !j.record)
        return SLLG_E_STATE;
    if (m_series)
        std::memcpy(m_series, j.m_series.data(), j.m_series.size() * sizeof(double));
    if (E_series)
        std::memcpy(E_series, j.E_series.data(), j.E_series.size() * sizeof(double));
    return SLLG_OK;
}

sllg_status sllg_cancel(sllg_server* srv, uint64_t ticket)
{
    if (!srv)
        return SLLG_E_ARG;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->jobs.find(ticket);
        if (it == srv->jobs.end())
            return SLLG_E_ARG;
        if (settled(it->second->state))
            return SLLG_E_STATE;
        it->second->cancel = true;
    }
    srv->cv.notify_all();
    return SLLG_OK;
}

sllg_status sllg_release(sllg_server* srv, uint64_t ticket)
{
    if (!srv)
        return SLLG_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end())
        return SLLG_E_ARG;
    if (!settled(it->second->state))
        return SLLG_E_STATE;
    srv->jobs.erase(it);
    return SLLG_OK;
}

sllg_status sllg_server_get_stats(sllg_server* srv, sllg_server_stats* stats)
{
    if (!srv || !stats)
        return SLLG_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    *stats = srv->stats;
    stats->active = (int64_t)srv->active.size();
    stats->queued = (int64_t)srv->queue.size();
    return SLLG_OK;
}

}  // extern "C"
