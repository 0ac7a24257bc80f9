// C ABI of a single spin system (see include/sllg.h).  A system is a batch
// of one replica; host-side set-up is kept until the first call that needs
// the device, then uploaded once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sllg.h"
#include "batch.hpp"
#include "kernels.hpp"
#include "prepare.hpp"

using namespace sllg;

namespace {

// Fields of the replica record that the host loop edits, independent of the
// precision.
struct ReplicaDevBase {
    double** records;
    double** acc;
    int32_t* flags;
    int32_t* nsteps;
    int64_t* rec_pos;
    int64_t* avg_first;
    int64_t* avg_block_len;
    int32_t* avg_blocks;
};

thread_local std::string g_create_error;

constexpr int kAvgCap = 4096;           // most averaging blocks per call
constexpr int64_t kHostChunk = 1024;    // steps per chunk without graphs

// Precision-independent interface of the one-replica engine.
struct Engine {
    virtual ~Engine() = default;
    virtual void create(const HostStructure& s, const HostMaterials& m, const Dynamics& d,
                        const std::vector<double>& S, int64_t rec_cap) = 0;
    virtual void set_spins(const std::vector<double>& S) = 0;
    virtual void get_spins(double* out, hipStream_t st) = 0;
    virtual void set_dynamics(const HostStructure& s, const HostMaterials& m, const Dynamics& d) = 0;
    virtual ReplicaDevBase& rec() = 0;
    virtual void run_chunk(int K, hipStream_t st, bool graph) = 0;
    virtual void measure_now(hipStream_t st) = 0;
    virtual void set_remap(int v) = 0;
    virtual void set_grid_scale(double f) = 0;
    virtual void set_tile_order(int order, int group) = 0;
    virtual void set_window(bool on) = 0;
    virtual void mc_sweep(uint64_t step, double cone, double inv_kT, unsigned long long* accepted,
                          hipStream_t st) = 0;
    virtual void record_current(int slot, hipStream_t st) = 0;
    virtual double max_torque(hipStream_t st) = 0;
    virtual void demag_update(hipStream_t st) = 0;
    virtual void demag_fetch(std::vector<double>& out, hipStream_t st) = 0;
    virtual void demag_set(const std::vector<double>& in) = 0;
    virtual size_t spin_bytes() = 0;
    virtual void save_spins(void* dst, hipStream_t st) = 0;
    virtual void load_spins(const void* src, hipStream_t st) = 0;
    // non-finite-spin flag: read (waits for st), or copied into pinned host
    // memory on st
    virtual bool fault(hipStream_t st) = 0;
    virtual void fault_async(int32_t* host, hipStream_t st) = 0;
    virtual int parity() = 0;
    virtual void set_parity(int p) = 0;
    virtual void mark_dirty() = 0;           // the record mirror changed
    virtual void mark_scalars_dirty() = 0;   // only its step count or record flags changed
    virtual uint64_t step() = 0;
    virtual void set_step(uint64_t step) = 0;
    virtual int64_t rec_cap() = 0;
    // fused plane-marching step
    virtual void set_fused(bool on) = 0;
    virtual bool fused_capable() = 0;          // the replica can take the fused step
    virtual FusedShape fused_shape() = 0;
    virtual void set_fused_shape(const FusedShape& f) = 0;
    virtual std::vector<FusedShape> fused_candidates(int max_count) = 0;
    virtual size_t lds_limit() = 0;
};

}  // namespace

// Error text of the calls without a handle (sllg_last_error(NULL)); used by
// the host-side structure builders.
void sllg::set_create_error(const std::string& msg) { g_create_error = msg; }

namespace {

template <typename R>
struct EngineT final : Engine {
    explicit EngineT(int device) : batch(device, &alloc, 1) {}
    DirectAllocator alloc;
    Batch<R> batch;
    int q = -1;
    int64_t cap = 0;
    ReplicaDevBase view{};

    void bind()
    {
        ReplicaDev<R>& r = batch.mirror(q);
        view = ReplicaDevBase{&r.records, &r.acc, &r.flags, &r.nsteps, &r.rec_pos,
                              &r.avg_first, &r.avg_block_len, &r.avg_blocks};
    }
    void create(const HostStructure& s, const HostMaterials& m, const Dynamics& d,
                const std::vector<double>& S, int64_t rec_cap) override
    {
        q = batch.add(s, m, d, S, rec_cap, kAvgCap);
        cap = rec_cap;
        bind();
    }
    void set_spins(const std::vector<double>& S) override { batch.set_spins(q, S); }
    void get_spins(double* out, hipStream_t st) override { batch.get_spins(q, out, st); }
    void set_dynamics(const HostStructure& s, const HostMaterials& m, const Dynamics& d) override
    {
        ReplicaDev<R>& r = batch.mirror(q);
        const uint64_t step = r.step;   // the device-side counter is authoritative
        Dynamics dd = d;
        dd.step = step;
        fill_parameters(r, s, m, dd);
        batch.upload_materials(q, m, dd);
        batch.mark_dirty();
    }
    ReplicaDevBase& rec() override { return view; }
    void run_chunk(int K, hipStream_t st, bool graph) override { batch.run_chunk(K, st, graph); }
    void measure_now(hipStream_t st) override { batch.measure_now(st); }
    void set_remap(int v) override { batch.set_remap(v); }
    void set_grid_scale(double f) override { batch.set_grid_scale(f); }
    void set_tile_order(int order, int group) override { batch.set_tile_order(order, group); }
    void set_window(bool on) override { batch.set_window(on); }
    void mc_sweep(uint64_t step, double cone, double inv_kT, unsigned long long* accepted,
                  hipStream_t st) override
    {
        batch.mc_sweep(q, step, cone, inv_kT, accepted, st);
    }
    void record_current(int slot, hipStream_t st) override { batch.record_current(slot, st); }
    void demag_update(hipStream_t st) override { batch.demag_update(q, st); }
    void demag_fetch(std::vector<double>& out, hipStream_t st) override { batch.demag_fetch(q, out, st); }
    void demag_set(const std::vector<double>& in) override { batch.demag_set(q, in); }
    double max_torque(hipStream_t st) override
    {
        std::vector<double> t;
        batch.max_torque(t, st);
        return t[(size_t)q];
    }
    size_t spin_bytes() override { return 3 * (size_t)batch.mirror(q).n * sizeof(R); }
    void save_spins(void* dst, hipStream_t st) override { batch.save_spins(q, dst, st); }
    void load_spins(const void* src, hipStream_t st) override { batch.load_spins(q, src, st); }
    bool fault(hipStream_t st) override { return batch.fault(q, st); }
    void fault_async(int32_t* host, hipStream_t st) override { batch.fault_async(q, host, st); }
    int parity() override { return batch.mirror(q).parity; }
    void set_parity(int p) override
    {
        batch.mirror(q).parity = p;
        batch.mark_dirty();
    }
    void mark_dirty() override { batch.mark_dirty(); }
    void mark_scalars_dirty() override { batch.mark_scalars_dirty(); }
    uint64_t step() override { return batch.mirror(q).step; }
    void set_step(uint64_t step) override
    {
        batch.mirror(q).step = step;
        batch.mark_dirty();
    }
    int64_t rec_cap() override { return cap; }
    void set_fused(bool on) override { batch.set_fused(on); }
    bool fused_capable() override
    {
        return (batch.mirror(q).flags & kFused) && batch.mirror(q).f_partials;
    }
    FusedShape fused_shape() override { return batch.fused_shape(q); }
    void set_fused_shape(const FusedShape& f) override { batch.set_fused_shape(q, f); }
    size_t lds_limit() override { return batch.lds_limit(); }
    std::vector<FusedShape> fused_candidates(int max_count) override
    {
        if (!batch.mirror(q).f_partials)
            return {};
        return batch.fused_candidate_shapes(q, max_count);
    }
};

}  // namespace

struct sllg_system {
    int device = 0;
    sllg_precision prec = SLLG_FP32;
    int64_t n = 0;
    std::string err;
    bool has_nb = false, has_mat = false, has_int = false;
    HostStructure st;
    HostMaterials mat;
    Dynamics dyn;
    std::vector<double> spins;       // host state until the engine exists
    // the caller's material arrays, kept so that the cubic anisotropy can
    // be combined with them whichever is set last
    std::vector<double> in_mu, in_ku, in_axis, in_kc;
    int in_per_site = 0, in_kc_per_site = 0;
    // the demagnetising field on the device belongs to the current state
    // and schedule; false: recompute before the next step that needs it
    bool demag_valid = false;
    // a held field restored from a checkpoint before the engine exists
    std::vector<double> demag_pending;
    int64_t opt_check_symmetry = 1;
    int64_t opt_graph_steps = -1;    // -1 = automatic
    int64_t opt_xcd_remap = 1;
    int64_t opt_grid_scale_pct = 100;   // workgroups per launch, % of the resident grid
    int64_t opt_tile_order = 1;         // plane-swept column groups when a plane stride is found
    int64_t opt_tile_group = 0;         // tile columns per group, 0 = from the L2 size
    int64_t opt_tile_sites = 0;         // sites per tile, 0 = from the system size
    int64_t opt_lds_window = 1;         // neighbours through the LDS tile window (1) or all from HBM (0)
    bool tuned = false;
    double tuned_us = 0.0;
    int64_t opt_stencil = 1;
    int64_t opt_mc_colouring = 0;       // Monte Carlo colouring visits: 0 ascending sites, 1 basis site and cell parity
    int64_t opt_fused = 1;              // fused step: 0 never, 1 large systems, 2 whenever the lattice allows it
    FusedShape opt_fshape;              // all fields > 0: this shape instead of the model's
    hipStream_t own = nullptr;
    std::unique_ptr<Engine> eng;
    std::vector<double> staging;
    unsigned long long* d_mc_acc = nullptr;   // accepted trials per Monte Carlo step (device)
    int64_t mc_acc_cap = 0;
    // the non-finite-spin flag as the last sllg_integrate_dev left it:
    // copied into pinned memory on its stream, valid once fault_ev completes
    int32_t* fault_host = nullptr;
    hipEvent_t fault_ev = nullptr;
};

namespace {

sllg_status guard(sllg_system* sys, const std::function<void()>& fn);

int64_t graph_steps(const sllg_system* s)
{
    if (s->opt_graph_steps >= 0)
        return s->opt_graph_steps & ~int64_t(1);
    return s->n < (int64_t(1) << 20) ? 64 : 0;
}

void ensure_device(sllg_system* s);
void require_ready(sllg_system* s);

// The caller's stream, or the library's own (opening the device if needed);
// every caller needs a fully set-up system.
hipStream_t pick_stream(sllg_system* s, void* stream)
{
    require_ready(s);
    ensure_device(s);
    return stream ? (hipStream_t)stream : s->own;
}

void require_ready(sllg_system* s)
{
    if (!s->has_nb)
        fail(SLLG_E_STATE, "neighbour list not set (sllg_set_neighbours)");
    if (!s->has_mat)
        fail(SLLG_E_STATE, "materials not set (sllg_set_materials)");
    if (!s->has_int)
        fail(SLLG_E_STATE, "integrator not set (sllg_set_integrator)");
}

// The device is checked and the library stream created at the first call
// that needs the GPU, so host-side set-up and validation work without one.
void ensure_device(sllg_system* s)
{
    if (s->own)
        return;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || s->device >= count)
        fail(SLLG_E_DEVICE, "HIP device " + std::to_string(s->device) + " is not available");
    hip_check(hipSetDevice(s->device), "hipSetDevice");
    hip_check(hipStreamCreateWithFlags(&s->own, hipStreamNonBlocking), "hipStreamCreate");
}

// Spins from which the fused step is the default (below it the two-launch
// step's shallow launches win: measured on bcc blocks, 0.52M spins 24.0
// against 21.2 us per step, 1.77M spins 40.8 against 52.4 us).
constexpr int64_t kFusedMinSpins = int64_t(1) << 20;

bool fused_wanted(const sllg_system* s)
{
    return s->opt_fused == 2 || (s->opt_fused == 1 && s->n >= kFusedMinSpins);
}

Engine& engine(sllg_system* s)
{
    require_ready(s);
    ensure_device(s);
    if (!s->eng) {
        hip_check(hipSetDevice(s->device), "hipSetDevice");
        if (s->prec == SLLG_FP32)
            s->eng = std::make_unique<EngineT<float>>(s->device);
        else
            s->eng = std::make_unique<EngineT<double>>(s->device);
        const int64_t G = graph_steps(s);
        s->eng->create(s->st, s->mat, s->dyn, s->spins, std::max<int64_t>(G, kHostChunk));
        s->eng->set_remap((int)s->opt_xcd_remap);
        s->eng->set_grid_scale(s->opt_grid_scale_pct / 100.0);
        s->eng->set_tile_order((int)s->opt_tile_order, (int)s->opt_tile_group);
        s->eng->set_window(s->opt_lds_window != 0);
        s->eng->set_fused(fused_wanted(s));
        const FusedShape& f = s->opt_fshape;
        if (f.px > 0 && f.py > 0 && f.planes > 0 && f.bt > 0 && s->eng->fused_capable())
            s->eng->set_fused_shape(f);
        if (s->st.demag.on && s->demag_valid && !s->demag_pending.empty())
            s->eng->demag_set(s->demag_pending);
        s->demag_pending.clear();
    }
    hip_check(hipSetDevice(s->device), "hipSetDevice");
    return *s->eng;
}

// Tear the engine down after a structural change, keeping the spins and the
// step counter.
void drop_engine(sllg_system* s)
{
    if (!s->eng)
        return;
    s->spins.assign(3 * (size_t)s->n, 0.0);
    s->eng->get_spins(s->spins.data(), s->own);
    s->dyn.step = s->eng->step();
    // a held demagnetising field stays in effect across the rebuild
    s->demag_pending.clear();
    if (s->st.demag.on && s->demag_valid)
        s->eng->demag_fetch(s->demag_pending, s->own);
    s->eng.reset();
}

// The demagnetising field for the step about to run: recomputed from the
// current state when the step number is a multiple of the update interval
// or no field is held.  Returns the steps that may run before the next
// update (n_steps when there is no demagnetising field).
int64_t demag_before_steps(sllg_system* s, Engine& e, int64_t n_steps, hipStream_t st)
{
    const HostDemag& dm = s->st.demag;
    if (!dm.on)
        return n_steps;
    const uint64_t k = e.step();
    const int64_t into = (int64_t)(k % (uint64_t)dm.every);
    if (!s->demag_valid || into == 0) {
        e.demag_update(st);
        s->demag_valid = true;
    }
    return std::min<int64_t>(n_steps, dm.every - into);
}

sllg_status guard(sllg_system* sys, const std::function<void()>& fn)
{
    if (!sys)
        return SLLG_E_ARG;
    try {
        fn();
        sys->err.clear();
        return SLLG_OK;
    } catch (const Failure& f) {
        sys->err = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        sys->err = "host allocation failed";
        return SLLG_E_NOMEM;
    } catch (const std::exception& e) {
        sys->err = e.what();
        return SLLG_E_DEVICE;
    } catch (...) {
        sys->err = "unknown failure";
        return SLLG_E_DEVICE;
    }
}

// Advance n steps in chunks; records (m, E) of each step go to the host
// arrays and/or the device arrays given.
void run_steps(sllg_system* s, int64_t n_steps, double* m_out, double* E_out, double* m_dev,
               double* E_dev, hipStream_t st, int32_t extra_flags)
{
    Engine& e = engine(s);
    ReplicaDevBase& r = e.rec();
    const bool host_rec = m_out || E_out;
    const bool dev_rec = m_dev || E_dev;
    const bool record = host_rec || dev_rec || (extra_flags & kAverage);
    const int64_t G = graph_steps(s);
    const int64_t chunk = G > 0 ? G : std::min<int64_t>(kHostChunk, e.rec_cap());
    const int32_t flags =
        (*r.flags & ~(kRecord | kRecordSeries | kAverage)) | (record ? kRecord : 0) | extra_flags;
    if (flags != *r.flags || *r.rec_pos != 0) {
        *r.flags = flags;
        *r.rec_pos = 0;
        e.mark_scalars_dirty();
    }
    int64_t done = 0;
    bool bad = false;
    while (done < n_steps) {
        const int64_t ns = demag_before_steps(s, e, std::min<int64_t>(chunk, n_steps - done), st);
        if (*r.nsteps != (int32_t)ns || *r.flags != flags) {
            *r.nsteps = (int32_t)ns;
            *r.flags = flags;
            e.mark_scalars_dirty();
        }
        const bool use_graph = G > 0 && ns == G;
        e.run_chunk((int)(use_graph ? G : ns), st, use_graph);
        if (dev_rec)
            hip_check(launch_scatter_records(*r.records, (int)ns, m_dev ? m_dev + 3 * done : nullptr,
                                             E_dev ? E_dev + done : nullptr, st),
                      "scatter records");
        if (host_rec) {
            s->staging.resize(4 * (size_t)ns);
            hip_check(hipMemcpyAsync(s->staging.data(), *r.records, 32 * (size_t)ns, hipMemcpyDeviceToHost, st),
                      "download records");
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            for (int64_t t = 0; t < ns; ++t) {
                const double* rec = &s->staging[4 * (size_t)t];
                if (m_out) {
                    m_out[3 * (done + t)] = rec[0];
                    m_out[3 * (done + t) + 1] = rec[1];
                    m_out[3 * (done + t) + 2] = rec[2];
                }
                if (E_out)
                    E_out[done + t] = rec[3];
                if (!std::isfinite(rec[3]))
                    bad = true;
            }
        }
        done += ns;
    }
    if (bad)
        fail(SLLG_E_NUMERIC, "the energy became non-finite during integration");
}

// Monte Carlo steps ("Monte Carlo Methods"): each step sweeps every colour
// class once; records of m and E after each step, accepted trials per step.
void mc_steps(sllg_system* s, int64_t n_steps, double* m_out, double* E_out, int64_t* acc_out,
              hipStream_t st)
{
    if (s->st.demag.on)
        fail(SLLG_E_STATE, "Monte Carlo with the demagnetising field is not supported");
    Engine& e = engine(s);
    ReplicaDevBase& r = e.rec();
    const bool record = m_out || E_out;
    const double T = s->dyn.temperature;
    const double cone = 2.0 / 25.0 * std::pow(kBoltzmann * T / kBohrMagneton, 0.2);
    const double inv_kT = T > 0.0 ? 1.0 / (kBoltzmann * T) : 0.0;
    const int64_t chunk = std::min<int64_t>(kHostChunk, e.rec_cap());
    const int32_t saved_flags = *r.flags;
    const int32_t saved_nsteps = *r.nsteps;
    // the measuring pass sweeps the replica's tiles: it takes part with nsteps 1
    *r.flags = (saved_flags & ~(kRecord | kRecordSeries | kAverage)) | (record ? kRecord : 0);
    *r.nsteps = 1;
    *r.rec_pos = 0;
    e.mark_dirty();
    if (s->mc_acc_cap < chunk) {   // kept for the system's lifetime
        if (s->d_mc_acc) {
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            hip_check(hipFree(s->d_mc_acc), "hipFree(accepted)");
            s->d_mc_acc = nullptr;
            s->mc_acc_cap = 0;
        }
        hip_check(hipMalloc(&s->d_mc_acc, sizeof(unsigned long long) * (size_t)chunk), "hipMalloc(accepted)");
        s->mc_acc_cap = chunk;
    }
    unsigned long long* d_acc = s->d_mc_acc;
    std::vector<unsigned long long> acc((size_t)chunk);
    const uint64_t step0 = e.step();
    bool bad = false;
    {
        for (int64_t done = 0; done < n_steps;) {
            const int64_t ns = std::min<int64_t>(chunk, n_steps - done);
            hip_check(hipMemsetAsync(d_acc, 0, sizeof(unsigned long long) * (size_t)ns, st), "clear counts");
            for (int64_t t = 0; t < ns; ++t) {
                e.mc_sweep(step0 + (uint64_t)(done + t), cone, inv_kT, d_acc + t, st);
                if (record)
                    e.record_current((int)t, st);
            }
            hip_check(hipMemcpyAsync(acc.data(), d_acc, sizeof(unsigned long long) * (size_t)ns,
                                     hipMemcpyDeviceToHost, st),
                      "download counts");
            if (record) {
                s->staging.resize(4 * (size_t)ns);
                hip_check(hipMemcpyAsync(s->staging.data(), *r.records, 32 * (size_t)ns, hipMemcpyDeviceToHost,
                                         st),
                          "download records");
            }
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            for (int64_t t = 0; t < ns; ++t) {
                if (acc_out)
                    acc_out[done + t] = (int64_t)acc[(size_t)t];
                if (!record)
                    continue;
                const double* rec = &s->staging[4 * (size_t)t];
                if (m_out) {
                    m_out[3 * (done + t)] = rec[0];
                    m_out[3 * (done + t) + 1] = rec[1];
                    m_out[3 * (done + t) + 2] = rec[2];
                }
                if (E_out)
                    E_out[done + t] = rec[3];
                if (!std::isfinite(rec[3]))
                    bad = true;
            }
            done += ns;
        }
    }
    *r.flags = saved_flags;
    *r.nsteps = saved_nsteps;
    e.set_step(step0 + (uint64_t)n_steps);
    e.mark_dirty();
    if (bad)
        fail(SLLG_E_NUMERIC, "the energy became non-finite during Monte Carlo");
    if (n_steps > 0 && e.fault(st))
        fail(SLLG_E_NUMERIC, "a trial spin became non-finite during Monte Carlo (the state is kept)");
}

void measure_state(sllg_system* s, double m[3], double* E, hipStream_t st)
{
    Engine& e = engine(s);
    ReplicaDevBase& r = e.rec();
    const int32_t saved = *r.flags;
    *r.flags = (saved & ~(kRecordSeries | kAverage)) | kRecord;
    *r.rec_pos = 0;
    e.mark_dirty();
    e.measure_now(st);
    double rec[4];
    hip_check(hipMemcpy(rec, *r.records, sizeof(rec), hipMemcpyDeviceToHost), "download record");
    if (m) {
        m[0] = rec[0];
        m[1] = rec[1];
        m[2] = rec[2];
    }
    if (E)
        *E = rec[3];
    *r.flags = saved;
    e.mark_dirty();
    if (!std::isfinite(rec[3]))
        fail(SLLG_E_NUMERIC, "the energy of the current state is not finite");
}

void average(sllg_system* s, int64_t n_eq, int64_t n_avg, int n_blocks, double out[8], hipStream_t st)
{
    if (n_eq < 0 || n_avg < 1)
        fail(SLLG_E_ARG, "need n_eq >= 0 and n_avg >= 1");
    if (n_blocks < 2 || n_blocks > kAvgCap || n_blocks > n_avg)
        fail(SLLG_E_ARG, "n_blocks must be in 2..min(n_avg, 4096)");
    if (!out)
        fail(SLLG_E_ARG, "out must not be NULL");
    Engine& e = engine(s);
    ReplicaDevBase& r = e.rec();
    const int64_t block_len = n_avg / n_blocks;
    hip_check(hipMemsetAsync(*r.acc, 0, sizeof(double) * 5 * (size_t)n_blocks, st), "clear sums");
    run_steps(s, n_eq, nullptr, nullptr, nullptr, nullptr, st, 0);
    *r.avg_first = (int64_t)e.step();
    *r.avg_block_len = block_len;
    *r.avg_blocks = n_blocks;
    e.mark_dirty();
    run_steps(s, n_avg, nullptr, nullptr, nullptr, nullptr, st, kAverage);
    std::vector<double> acc(5 * (size_t)n_blocks);
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    hip_check(hipMemcpy(acc.data(), *r.acc, acc.size() * sizeof(double), hipMemcpyDeviceToHost),
              "download sums");
    *r.flags &= ~kAverage;
    e.mark_dirty();
    averages_from_block_sums(acc.data(), n_blocks, block_len, out);
    if (!std::isfinite(out[5]))
        fail(SLLG_E_NUMERIC, "the energy became non-finite during averaging");
}

// Monte Carlo thermal average: n_eq steps, then n_avg steps with m and E
// taken after every step, summed per block on the host in step order.
void mc_average(sllg_system* s, int64_t n_eq, int64_t n_avg, int n_blocks, double out[9], hipStream_t st)
{
    if (n_eq < 0 || n_avg < 1)
        fail(SLLG_E_ARG, "need n_eq >= 0 and n_avg >= 1");
    if (n_blocks < 2 || n_blocks > kAvgCap || n_blocks > n_avg)
        fail(SLLG_E_ARG, "n_blocks must be in 2..min(n_avg, 4096)");
    if (!out)
        fail(SLLG_E_ARG, "out must not be NULL");
    mc_steps(s, n_eq, nullptr, nullptr, nullptr, st);
    const int64_t block_len = n_avg / n_blocks;
    std::vector<double> sums(5 * (size_t)n_blocks, 0.0);
    constexpr int64_t kPiece = 4096;
    std::vector<double> m(3 * (size_t)std::min(kPiece, n_avg)), E((size_t)std::min(kPiece, n_avg));
    std::vector<int64_t> acc((size_t)std::min(kPiece, n_avg));
    double accepted = 0.0;
    for (int64_t done = 0; done < n_avg;) {
        const int64_t ns = std::min(kPiece, n_avg - done);
        mc_steps(s, ns, m.data(), E.data(), acc.data(), st);
        for (int64_t t = 0; t < ns; ++t) {
            accepted += (double)acc[(size_t)t];
            const int64_t k = done + t;
            if (k >= block_len * n_blocks)
                continue;
            double* b = &sums[5 * (size_t)(k / block_len)];
            const double* mt = &m[3 * (size_t)t];
            b[0] += std::sqrt(mt[0] * mt[0] + mt[1] * mt[1] + mt[2] * mt[2]);
            b[1] += mt[0];
            b[2] += mt[1];
            b[3] += mt[2];
            b[4] += E[(size_t)t];
        }
        done += ns;
    }
    averages_from_block_sums(sums.data(), n_blocks, block_len, out);
    out[8] = accepted / ((double)s->n * (double)n_avg);
}

// Launch-shape autotuner: time each candidate over a few steps of the real
// system and keep the fastest.  With the fused step active: the model's
// eight best fused shapes (tile, planes per item, block size); else the
// two-launch step's launch shapes
// (XCD-contiguous tile ranges or not; workgroups per launch as 1/2, 1 or 2
// resident grids; tile order; LDS window).  Small systems also try the
// steps per captured graph.  Results do not depend on these choices, and the
// spins, step counter and buffer parity are restored afterwards, so tuning
// leaves the trajectory untouched.
double autotune(sllg_system* s, int trial_steps, hipStream_t st)
{
    Engine& e = engine(s);
    ReplicaDevBase& r = e.rec();
    const uint64_t step0 = e.step();
    const int par0 = e.parity();
    void* saved = nullptr;
    hip_check(hipMalloc(&saved, e.spin_bytes()), "hipMalloc(autotune)");
    struct Cand {
        int remap;
        int64_t scale_pct;
        int64_t graph;
        int64_t order;
        int64_t window;
        int64_t fused;       // 1: the fused step in shape fs
        FusedShape fs;
    };
    std::vector<Cand> cands;
    const bool small = s->n < (int64_t(1) << 20);
    const std::vector<int64_t> graphs = small ? std::vector<int64_t>{64, 16, 256} : std::vector<int64_t>{0};
    const bool fusable = fused_wanted(s) && e.fused_capable();
    if (fusable) {
        // the model's best fused shapes (the spins do not depend on the shape)
        // FP64: more of them (the model ranks FP64 shapes less sharply)
        for (const FusedShape& f : e.fused_candidates(s->prec == SLLG_FP64 ? 12 : 8))
            for (int64_t g : graphs)
                cands.push_back({1, 100, g, 1, 1, 1, f});
    } else {
        for (int64_t window : {1, 0})
            for (int64_t order : {1, 0})
                for (int remap : {1, 2, 0})
                    for (int64_t scale : {100, 50, 200})
                        for (int64_t g : graphs)
                            cands.push_back({remap, scale, g, order, window, 0, FusedShape{}});
    }
    hipEvent_t a = nullptr, b = nullptr;
    double best = 1e30;
    Cand best_c = {(int)s->opt_xcd_remap, s->opt_grid_scale_pct, graph_steps(s), s->opt_tile_order,
                   s->opt_lds_window, fusable ? 1 : 0, fusable ? e.fused_shape() : FusedShape{}};
    auto apply = [&](const Cand& c) {
        s->opt_xcd_remap = c.remap;
        s->opt_grid_scale_pct = c.scale_pct;
        s->opt_graph_steps = c.graph;
        s->opt_tile_order = c.order;
        s->opt_lds_window = c.window;
        e.set_remap(c.remap);
        e.set_grid_scale(c.scale_pct / 100.0);
        e.set_tile_order((int)c.order, (int)s->opt_tile_group);
        e.set_window(c.window != 0);
        if (c.fused) {
            s->opt_fshape = c.fs;
            e.set_fused_shape(c.fs);
        }
    };
    const int32_t flags0 = *r.flags;
    // the held demagnetising field belongs to the trajectory: kept aside and
    // put back, so the schedule continues as if no trial had run
    const bool demag_valid0 = s->demag_valid;
    std::vector<double> demag0;
    if (s->st.demag.on && demag_valid0)
        e.demag_fetch(demag0, st);
    const char* log_env = std::getenv("SLLG_AUTOTUNE_LOG");   // print every candidate's time
    const bool log = log_env && *log_env && *log_env != '0';
    try {
        hip_check(hipEventCreate(&a), "hipEventCreate");
        hip_check(hipEventCreate(&b), "hipEventCreate");
        e.save_spins(saved, st);
        run_steps(s, std::max(trial_steps, 8), nullptr, nullptr, nullptr, nullptr, st, 0);   // first touch
        for (const Cand& c : cands) {
            if (c.graph > e.rec_cap())
                continue;
            apply(c);
            const int steps = c.graph > 0 ? (int)std::max<int64_t>(c.graph, trial_steps) : trial_steps;
            run_steps(s, std::max<int64_t>(c.graph, 2), nullptr, nullptr, nullptr, nullptr, st, 0);  // warm
            double us = 1e30;
            for (int rep = 0; rep < 2; ++rep) {   // best of two
                hip_check(hipEventRecord(a, st), "hipEventRecord");
                run_steps(s, steps, nullptr, nullptr, nullptr, nullptr, st, 0);
                hip_check(hipEventRecord(b, st), "hipEventRecord");
                hip_check(hipEventSynchronize(b), "hipEventSynchronize");
                float ms = 0.f;
                hip_check(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
                us = std::min(us, 1e3 * ms / steps);
            }
            if (log && c.fused)
                std::fprintf(stderr, "[sllg autotune] fused tile %d x %d, %d planes, %d threads, graph %lld: %.1f us/step\n",
                             c.fs.px - 2, c.fs.py - 2, c.fs.planes, c.fs.bt, (long long)c.graph, us);
            else if (log)
                std::fprintf(stderr,
                             "[sllg autotune] lds_window %lld xcd_remap %d grid %lld%% graph %lld tile_order %lld: "
                             "%.1f us/step\n",
                             (long long)c.window, c.remap, (long long)c.scale_pct, (long long)c.graph,
                             (long long)c.order, us);
            if (us < best) {
                best = us;
                best_c = c;
            }
        }
    } catch (...) {
        (void)hipFree(saved);
        if (a)
            (void)hipEventDestroy(a);
        if (b)
            (void)hipEventDestroy(b);
        throw;
    }
    // restore the state and apply the winner
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    e.set_parity(par0);
    e.load_spins(saved, st);
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    e.set_step(step0);
    *r.flags = flags0;
    e.mark_dirty();
    if (s->st.demag.on) {
        if (demag_valid0)
            e.demag_set(demag0);
        s->demag_valid = demag_valid0;
    }
    (void)hipFree(saved);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    apply(best_c);
    s->tuned = true;
    s->tuned_us = best;
    return best;
}

// The fused shape in use (engine), requested (option), or 0 when unknown.
FusedShape current_fused_shape(const sllg_system* s)
{
    if (s->eng && s->eng->fused_capable())
        return s->eng->fused_shape();
    return s->opt_fshape;
}

// The next integration takes the fused step: a lattice it takes in the
// system's precision (FP64: the compiled kinds), uniform materials, scalar
// exchange, no cubic anisotropy or demagnetising field, and the option on.
bool fused_will_run(const sllg_system* s)
{
    return fused_wanted(s) && fused_precision_ok(s->st.lat, s->n, s->prec == SLLG_FP32 ? 4 : 8) && s->has_mat &&
           !s->mat.per_site_material && !s->mat.per_site_axis && !s->st.tensor && !s->mat.cubic && !s->st.demag.on;
}

void apply_dynamics(sllg_system* s)
{
    if (s->eng)
        s->eng->set_dynamics(s->st, s->mat, s->dyn);
}

}  // namespace

extern "C" {

const char* sllg_status_string(sllg_status status)
{
    switch (status) {
    case SLLG_OK: return "SLLG_OK";
    case SLLG_E_ARG: return "SLLG_E_ARG";
    case SLLG_E_NOMEM: return "SLLG_E_NOMEM";
    case SLLG_E_DEVICE: return "SLLG_E_DEVICE";
    case SLLG_E_STATE: return "SLLG_E_STATE";
    case SLLG_E_BUDGET: return "SLLG_E_BUDGET";
    case SLLG_E_NUMERIC: return "SLLG_E_NUMERIC";
    case SLLG_E_CANCELLED: return "SLLG_E_CANCELLED";
    }
    return "unknown status";
}

sllg_status sllg_create(int device, sllg_precision precision, int64_t n_spins, sllg_system** out)
{
    if (!out) {
        g_create_error = "out must not be NULL";
        return SLLG_E_ARG;
    }
    *out = nullptr;
    if (precision != SLLG_FP32 && precision != SLLG_FP64) {
        g_create_error = "precision must be SLLG_FP32 or SLLG_FP64";
        return SLLG_E_ARG;
    }
    if (n_spins < 1 || n_spins >= (int64_t(1) << kColBits)) {
        g_create_error = "n_spins must be in 1 .. 2^28-1";
        return SLLG_E_ARG;
    }
    if (device < 0) {
        g_create_error = "device must be >= 0";
        return SLLG_E_ARG;
    }
    auto* s = new (std::nothrow) sllg_system();
    if (!s) {
        g_create_error = "host allocation failed";
        return SLLG_E_NOMEM;
    }
    s->device = device;
    s->prec = precision;
    s->n = n_spins;
    s->spins.assign(3 * (size_t)n_spins, 0.0);
    for (int64_t i = 0; i < n_spins; ++i)
        s->spins[3 * i + 2] = 1.0;
    g_create_error.clear();
    *out = s;
    return SLLG_OK;
}

void sllg_destroy(sllg_system* sys)
{
    if (!sys)
        return;
    if (sys->own) {
        (void)hipSetDevice(sys->device);
        (void)hipStreamSynchronize(sys->own);
    }
    if (sys->d_mc_acc) {
        (void)hipDeviceSynchronize();
        (void)hipFree(sys->d_mc_acc);
    }
    if (sys->fault_ev) {
        (void)hipEventSynchronize(sys->fault_ev);
        (void)hipEventDestroy(sys->fault_ev);
    }
    if (sys->fault_host)
        (void)hipHostFree(sys->fault_host);
    sys->eng.reset();
    if (sys->own)
        (void)hipStreamDestroy(sys->own);
    delete sys;
}

const char* sllg_last_error(const sllg_system* sys)
{
    return sys ? sys->err.c_str() : g_create_error.c_str();
}

sllg_status sllg_set_neighbours(sllg_system* sys, const int64_t* row_ptr, const int32_t* col,
                                const uint8_t* ntype, const double* J, int n_types)
{
    return guard(sys, [&] {
        HostStructure st = build_structure(sys->n, row_ptr, col, ntype, J, n_types,
                                           sys->opt_check_symmetry != 0, kHaloCap, sys->opt_stencil != 0);
        st.tile_request = (int)sys->opt_tile_sites;
        build_colours(st, false);   // no lattice declared yet
        drop_engine(sys);
        sys->st = std::move(st);
        sys->has_nb = true;
    });
}

sllg_status sllg_set_lattice(sllg_system* sys, int n_basis, const int cells[3], const int periodic[3])
{
    return guard(sys, [&] {
        if (!sys->has_nb)
            fail(SLLG_E_STATE, "neighbour list not set (sllg_set_neighbours)");
        HostStructure st = sys->st;
        set_lattice(st, n_basis, cells, periodic);
        if (sys->opt_mc_colouring)
            build_colours(st, true);
        drop_engine(sys);   // rebuilt at the next run with the fused step's buffers, state kept
        sys->st = std::move(st);
    });
}

namespace {

void install_materials(sllg_system* sys, HostMaterials m)
{
    if (sys->eng && m.per_site_material == sys->mat.per_site_material &&
        m.per_site_axis == sys->mat.per_site_axis && !m.per_site_material && !m.per_site_axis &&
        m.mat_mu.size() == sys->mat.mat_mu.size() && m.cubic == sys->mat.cubic) {
        sys->mat = std::move(m);
        apply_dynamics(sys);   // uniform materials: a table update suffices
    } else {
        drop_engine(sys);
        sys->mat = std::move(m);
    }
}

}  // namespace

sllg_status sllg_set_materials(sllg_system* sys, const double* mu_s, const double* k_u,
                               const double* easy_axis, int per_site)
{
    return guard(sys, [&] {
        HostMaterials m = build_materials(sys->n, mu_s, k_u, easy_axis, per_site,
                                          sys->in_kc.empty() ? nullptr : sys->in_kc.data(), sys->in_kc_per_site);
        const size_t cnt = per_site ? (size_t)sys->n : 1;
        sys->in_mu.assign(mu_s, mu_s + cnt);
        sys->in_ku.assign(k_u, k_u + cnt);
        sys->in_axis.assign(easy_axis, easy_axis + 3 * cnt);
        sys->in_per_site = per_site;
        install_materials(sys, std::move(m));
        sys->has_mat = true;
    });
}

sllg_status sllg_set_cubic_anisotropy(sllg_system* sys, const double* k_c, int per_site)
{
    return guard(sys, [&] {
        if (!sys->has_mat)
            fail(SLLG_E_STATE, "materials not set (sllg_set_materials)");
        if (per_site != 0 && per_site != 1)
            fail(SLLG_E_ARG, "per_site must be 0 or 1");
        std::vector<double> kc;
        if (k_c)
            kc.assign(k_c, k_c + (per_site ? (size_t)sys->n : 1));
        HostMaterials m = build_materials(sys->n, sys->in_mu.data(), sys->in_ku.data(), sys->in_axis.data(),
                                          sys->in_per_site, kc.empty() ? nullptr : kc.data(), per_site);
        sys->in_kc = std::move(kc);
        sys->in_kc_per_site = per_site;
        install_materials(sys, std::move(m));
    });
}

sllg_status sllg_set_exchange_tensors(sllg_system* sys, const double* J, int n_types)
{
    return guard(sys, [&] {
        if (!sys->has_nb)
            fail(SLLG_E_STATE, "neighbour list not set (sllg_set_neighbours)");
        set_exchange_tensors(sys->st, J, n_types);   // validates before it changes anything
        drop_engine(sys);
    });
}

sllg_status sllg_set_integrator(sllg_system* sys, double alpha, double gamma, double dt)
{
    return guard(sys, [&] {
        Dynamics d = sys->dyn;
        d.alpha = alpha;
        d.gamma = gamma;
        d.dt = dt;
        check_dynamics(d);
        if (sys->eng)
            d.step = sys->eng->step();
        sys->dyn = d;
        sys->has_int = true;
        apply_dynamics(sys);
    });
}

sllg_status sllg_set_conditions(sllg_system* sys, double temperature, const double H_app[3])
{
    return guard(sys, [&] {
        if (!H_app)
            fail(SLLG_E_ARG, "H_app must not be NULL");
        Dynamics d = sys->dyn;
        d.temperature = temperature;
        d.H[0] = H_app[0];
        d.H[1] = H_app[1];
        d.H[2] = H_app[2];
        if (!(temperature >= 0.0) || !std::isfinite(temperature))
            fail(SLLG_E_ARG, "temperature must be finite and >= 0");
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(d.H[c]))
                fail(SLLG_E_ARG, "applied field must be finite");
        if (sys->eng)
            d.step = sys->eng->step();
        sys->dyn = d;
        if (sys->has_int)
            apply_dynamics(sys);
    });
}

sllg_status sllg_set_rng(sllg_system* sys, uint64_t seed, uint64_t step)
{
    return guard(sys, [&] {
        sys->dyn.seed = seed;
        sys->dyn.step = step;
        if (sys->eng) {
            // set_dynamics keeps the engine's counter; overwrite it explicitly
            sys->eng->set_dynamics(sys->st, sys->mat, sys->dyn);
            sys->eng->set_step(step);
        }
    });
}

sllg_status sllg_get_step(const sllg_system* sys, uint64_t* step)
{
    if (!sys || !step)
        return SLLG_E_ARG;
    *step = sys->eng ? sys->eng->step() : sys->dyn.step;
    return SLLG_OK;
}

namespace {
// A new state has no fault: forget the copy the last sllg_integrate_dev
// queued (after it has landed) as well as the device flag (set_spins).
void clear_fault_copy(sllg_system* s)
{
    if (s->fault_ev) {
        hip_check(hipEventSynchronize(s->fault_ev), "hipEventSynchronize");
        *s->fault_host = 0;
    }
}
}  // namespace

sllg_status sllg_set_spins(sllg_system* sys, const double* S)
{
    return guard(sys, [&] {
        std::vector<double> v = normalised_spins(sys->n, S);
        sys->demag_valid = false;
        clear_fault_copy(sys);
        if (sys->eng) {
            hip_check(hipSetDevice(sys->device), "hipSetDevice");
            sys->eng->set_spins(v);
        } else {
            sys->spins = std::move(v);
        }
    });
}

sllg_status sllg_get_spins(sllg_system* sys, double* S_out)
{
    return guard(sys, [&] {
        if (!S_out)
            fail(SLLG_E_ARG, "S_out must not be NULL");
        if (sys->eng) {
            hip_check(hipSetDevice(sys->device), "hipSetDevice");
            sys->eng->get_spins(S_out, sys->own);
        } else {
            std::memcpy(S_out, sys->spins.data(), sys->spins.size() * sizeof(double));
        }
    });
}

sllg_status sllg_integrate(sllg_system* sys, int64_t n_steps, double* m_out, double* E_out, void* stream)
{
    return guard(sys, [&] {
        if (n_steps < 0)
            fail(SLLG_E_ARG, "n_steps must be >= 0");
        hipStream_t st = pick_stream(sys, stream);
        run_steps(sys, n_steps, m_out, E_out, nullptr, nullptr, st, 0);
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        if (n_steps > 0 && engine(sys).fault(st))
            fail(SLLG_E_NUMERIC, "a spin became non-finite during integration (the state is kept)");
        if (!m_out && !E_out && n_steps > 0) {
            double E;
            measure_state(sys, nullptr, &E, st);
        }
    });
}

sllg_status sllg_integrate_dev(sllg_system* sys, int64_t n_steps, double* m_dev, double* E_dev, void* stream)
{
    return guard(sys, [&] {
        if (n_steps < 0)
            fail(SLLG_E_ARG, "n_steps must be >= 0");
        // a non-finite spin left by an earlier call whose work has finished
        // (not waited for: the call stays asynchronous)
        if (sys->fault_ev && hipEventQuery(sys->fault_ev) == hipSuccess && *sys->fault_host)
            fail(SLLG_E_NUMERIC, "a spin became non-finite during an earlier sllg_integrate_dev call (the state is "
                                 "kept)");
        hipStream_t st = pick_stream(sys, stream);
        run_steps(sys, n_steps, nullptr, nullptr, m_dev, E_dev, st, 0);
        if (n_steps > 0) {
            if (!sys->fault_host) {
                hip_check(hipHostMalloc((void**)&sys->fault_host, sizeof(int32_t), hipHostMallocDefault),
                          "hipHostMalloc(fault flag)");
                *sys->fault_host = 0;
                hip_check(hipEventCreateWithFlags(&sys->fault_ev, hipEventDisableTiming), "hipEventCreate");
            }
            engine(sys).fault_async(sys->fault_host, st);
            hip_check(hipEventRecord(sys->fault_ev, st), "hipEventRecord");
        }
    });
}

sllg_status sllg_measure(sllg_system* sys, double m[3], double* E, void* stream)
{
    return guard(sys, [&] { measure_state(sys, m, E, pick_stream(sys, stream)); });
}

sllg_status sllg_mc(sllg_system* sys, int64_t n_steps, double* m_out, double* E_out, int64_t* accepted_out,
                    void* stream)
{
    return guard(sys, [&] {
        if (n_steps < 0)
            fail(SLLG_E_ARG, "n_steps must be >= 0");
        if (sys->st.demag.on)
            fail(SLLG_E_STATE, "Monte Carlo with the demagnetising field is not supported");
        if (n_steps > 0)
            mc_steps(sys, n_steps, m_out, E_out, accepted_out, pick_stream(sys, stream));
    });
}

sllg_status sllg_mc_average(sllg_system* sys, int64_t n_eq, int64_t n_avg, int n_blocks, double out[9],
                            void* stream)
{
    return guard(sys, [&] { mc_average(sys, n_eq, n_avg, n_blocks, out, pick_stream(sys, stream)); });
}

sllg_status sllg_average(sllg_system* sys, int64_t n_eq, int64_t n_avg, int n_blocks, double out[8],
                         void* stream)
{
    return guard(sys, [&] { average(sys, n_eq, n_avg, n_blocks, out, pick_stream(sys, stream)); });
}

sllg_status sllg_sweep_temperature(sllg_system* sys, const double* T, int64_t n_points, int64_t n_eq,
                                   int64_t n_avg, int n_blocks, double* out, void* stream)
{
    return guard(sys, [&] {
        if (!T || !out || n_points < 0)
            fail(SLLG_E_ARG, "T and out must not be NULL");
        for (int64_t k = 0; k < n_points; ++k)
            if (!(T[k] >= 0.0) || !std::isfinite(T[k]))
                fail(SLLG_E_ARG, "temperatures must be finite and >= 0");
        hipStream_t st = pick_stream(sys, stream);
        for (int64_t k = 0; k < n_points; ++k) {
            Engine& e = engine(sys);
            sys->dyn.temperature = T[k];
            sys->dyn.step = e.step();
            apply_dynamics(sys);
            average(sys, n_eq, n_avg, n_blocks, out + 8 * k, st);
        }
    });
}

sllg_status sllg_sweep_field(sllg_system* sys, const double* H, int64_t n_points, int64_t n_eq,
                             int64_t n_avg, int n_blocks, double* out, void* stream)
{
    return guard(sys, [&] {
        if (!H || !out || n_points < 0)
            fail(SLLG_E_ARG, "H and out must not be NULL");
        for (int64_t k = 0; k < 3 * n_points; ++k)
            if (!std::isfinite(H[k]))
                fail(SLLG_E_ARG, "fields must be finite");
        hipStream_t st = pick_stream(sys, stream);
        for (int64_t k = 0; k < n_points; ++k) {
            Engine& e = engine(sys);
            sys->dyn.H[0] = H[3 * k];
            sys->dyn.H[1] = H[3 * k + 1];
            sys->dyn.H[2] = H[3 * k + 2];
            sys->dyn.step = e.step();
            apply_dynamics(sys);
            average(sys, n_eq, n_avg, n_blocks, out + 8 * k, st);
        }
    });
}

namespace {

// Heun steps at T = 0 until the largest torque is at most tol (checked
// before the first step and after every check_every steps); returns the
// steps taken, or -1 when max_steps were taken first.  *torque: the last
// value checked.
void check_relax(const sllg_system* sys, double tol, int64_t max_steps, int64_t check_every)
{
    if (!(tol >= 0.0) || !std::isfinite(tol))
        fail(SLLG_E_ARG, "torque_tol must be finite and >= 0");
    if (max_steps < 0 || check_every < 1)
        fail(SLLG_E_ARG, "max_steps must be >= 0 and check_every >= 1");
    if (sys->dyn.temperature != 0.0)
        fail(SLLG_E_STATE, "relaxation needs T = 0 (the thermal field keeps the torque finite)");
}

int64_t relax(sllg_system* sys, double tol, int64_t max_steps, int64_t check_every, double* torque,
              hipStream_t st)
{
    check_relax(sys, tol, max_steps, check_every);
    Engine& e = engine(sys);
    int64_t taken = 0;
    if (sys->st.demag.on && !sys->demag_valid) {
        e.demag_update(st);
        sys->demag_valid = true;
    }
    double t = e.max_torque(st);
    while (t > tol) {
        if (taken >= max_steps) {
            *torque = t;
            return -1;
        }
        const int64_t ns = std::min(check_every, max_steps - taken);
        run_steps(sys, ns, nullptr, nullptr, nullptr, nullptr, st, 0);
        taken += ns;
        t = e.max_torque(st);
    }
    *torque = t;
    return taken;
}

}  // namespace

sllg_status sllg_max_torque(sllg_system* sys, double* torque_out, void* stream)
{
    return guard(sys, [&] {
        if (!torque_out)
            fail(SLLG_E_ARG, "torque_out must not be NULL");
        hipStream_t st = pick_stream(sys, stream);
        Engine& e = engine(sys);
        if (sys->st.demag.on && !sys->demag_valid) {
            e.demag_update(st);
            sys->demag_valid = true;
        }
        *torque_out = e.max_torque(st);
    });
}

sllg_status sllg_set_demag(sllg_system* sys, const double* pos, double cell_size, double atom_volume,
                           int64_t every)
{
    return guard(sys, [&] {
        if (!sys->has_nb)
            fail(SLLG_E_STATE, "neighbour list not set (sllg_set_neighbours)");
        HostDemag d;
        if (pos)
            d = build_demag(sys->n, pos, cell_size, atom_volume, every);
        drop_engine(sys);
        sys->st.demag = std::move(d);
        sys->demag_valid = false;
    });
}

sllg_status sllg_demag_field(sllg_system* sys, double* field_out, void* stream)
{
    return guard(sys, [&] {
        if (!field_out)
            fail(SLLG_E_ARG, "field_out must not be NULL");
        if (!sys->st.demag.on)
            fail(SLLG_E_STATE, "no demagnetising field set (sllg_set_demag)");
        hipStream_t st = pick_stream(sys, stream);
        Engine& e = engine(sys);
        // the field in effect: computed now only when none is held (the next
        // step would compute the same from the current state)
        if (!sys->demag_valid) {
            e.demag_update(st);
            sys->demag_valid = true;
        }
        std::vector<double> cells;
        e.demag_fetch(cells, st);
        const HostDemag& dm = sys->st.demag;
        for (int64_t i = 0; i < sys->n; ++i)
            for (int a = 0; a < 3; ++a)
                field_out[3 * i + a] = cells[3 * (size_t)dm.cell_of[(size_t)i] + a];
    });
}

sllg_status sllg_relax(sllg_system* sys, double torque_tol, int64_t max_steps, int64_t check_every,
                       int64_t* steps_out, double* torque_out, void* stream)
{
    sllg_status failed = SLLG_OK;
    const sllg_status st = guard(sys, [&] {
        check_relax(sys, torque_tol, max_steps, check_every);   // before the device is opened
        double t = 0.0;
        const int64_t n = relax(sys, torque_tol, max_steps, check_every, &t, pick_stream(sys, stream));
        if (steps_out)
            *steps_out = n;
        if (torque_out)
            *torque_out = t;
        if (n < 0)
            failed = SLLG_E_NUMERIC;
    });
    if (st == SLLG_OK && failed != SLLG_OK) {
        sys->err = "relaxation did not reach the torque tolerance within max_steps";
        return failed;
    }
    return st;
}

sllg_status sllg_hysteresis(sllg_system* sys, const double* H, int64_t n_points, double torque_tol,
                            int64_t max_steps, int64_t check_every, double* m_out, int64_t* steps_out,
                            void* stream)
{
    return guard(sys, [&] {
        if (!H || !m_out || n_points < 0)
            fail(SLLG_E_ARG, "H and m_out must not be NULL");
        for (int64_t k = 0; k < 3 * n_points; ++k)
            if (!std::isfinite(H[k]))
                fail(SLLG_E_ARG, "fields must be finite");
        check_relax(sys, torque_tol, max_steps, check_every);
        hipStream_t st = pick_stream(sys, stream);
        for (int64_t k = 0; k < n_points; ++k) {
            Engine& e = engine(sys);
            sys->dyn.H[0] = H[3 * k];
            sys->dyn.H[1] = H[3 * k + 1];
            sys->dyn.H[2] = H[3 * k + 2];
            sys->dyn.step = e.step();
            apply_dynamics(sys);
            double t = 0.0;
            const int64_t n = relax(sys, torque_tol, max_steps, check_every, &t, st);
            if (steps_out)
                steps_out[k] = n;
            double E;
            measure_state(sys, m_out + 3 * k, &E, st);
        }
    });
}

namespace {
struct CheckpointHeader {
    char magic[8];
    uint32_t version;
    uint32_t precision;
    int64_t n;
    uint64_t seed;
    uint64_t step;
};

// Version 2 adds the held demagnetising field: it belongs to the state
// (it was computed at the last update step and is held until the next), so
// a restored run continues exactly as the uninterrupted one.
struct CheckpointDemag {
    int64_t cells;       // cells of the field that follows (0: none held)
    int64_t reserved;
};

size_t demag_checkpoint_cells(const sllg_system* sys)
{
    return sys->st.demag.on && sys->demag_valid ? (size_t)sys->st.demag.cells : 0;
}
}  // namespace

sllg_status sllg_checkpoint_size(const sllg_system* sys, size_t* bytes)
{
    if (!sys || !bytes)
        return SLLG_E_ARG;
    *bytes = sizeof(CheckpointHeader) + sizeof(CheckpointDemag) + 3 * (size_t)sys->n * sizeof(double) +
             3 * demag_checkpoint_cells(sys) * sizeof(double);
    return SLLG_OK;
}

sllg_status sllg_checkpoint(sllg_system* sys, void* buf, size_t bytes)
{
    return guard(sys, [&] {
        size_t need = 0;
        sllg_checkpoint_size(sys, &need);
        if (!buf || bytes < need)
            fail(SLLG_E_ARG, "checkpoint buffer too small");
        CheckpointHeader h{};
        std::memcpy(h.magic, "SLLGCKP2", 8);
        h.version = 2;
        h.precision = (uint32_t)sys->prec;
        h.n = sys->n;
        h.seed = sys->dyn.seed;
        h.step = sys->eng ? sys->eng->step() : sys->dyn.step;
        CheckpointDemag d{};
        d.cells = (int64_t)demag_checkpoint_cells(sys);
        char* p = static_cast<char*>(buf);
        std::memcpy(p, &h, sizeof(h));
        std::memcpy(p + sizeof(h), &d, sizeof(d));
        double* S = reinterpret_cast<double*>(p + sizeof(h) + sizeof(d));
        if (sys->eng)
            sys->eng->get_spins(S, sys->own);
        else
            std::memcpy(S, sys->spins.data(), sys->spins.size() * sizeof(double));
        if (d.cells > 0) {
            std::vector<double> field;
            if (sys->eng)
                sys->eng->demag_fetch(field, sys->own);
            else
                field = sys->demag_pending;
            if (field.size() != 3 * (size_t)d.cells)
                fail(SLLG_E_STATE, "held demagnetising field missing");
            std::memcpy(S + 3 * (size_t)sys->n, field.data(), 3 * (size_t)d.cells * sizeof(double));
        }
    });
}

sllg_status sllg_restore(sllg_system* sys, const void* buf, size_t bytes)
{
    return guard(sys, [&] {
        CheckpointHeader h{};
        if (!buf || bytes < sizeof(h))
            fail(SLLG_E_ARG, "checkpoint buffer too small");
        std::memcpy(&h, buf, sizeof(h));
        const bool v1 = std::memcmp(h.magic, "SLLGCKP1", 8) == 0 && h.version == 1;
        const bool v2 = std::memcmp(h.magic, "SLLGCKP2", 8) == 0 && h.version == 2;
        if (!v1 && !v2)
            fail(SLLG_E_ARG, "not a checkpoint of this library");
        if (h.n != sys->n || h.precision != (uint32_t)sys->prec)
            fail(SLLG_E_ARG, "checkpoint is of a different system size or precision");
        CheckpointDemag d{};
        size_t off = sizeof(h);
        if (v2) {
            if (bytes < off + sizeof(d))
                fail(SLLG_E_ARG, "checkpoint truncated");
            std::memcpy(&d, static_cast<const char*>(buf) + off, sizeof(d));
            off += sizeof(d);
            if (d.cells < 0 || (d.cells > 0 && (!sys->st.demag.on || d.cells != sys->st.demag.cells)))
                fail(SLLG_E_ARG, "checkpoint holds a demagnetising field of another macrocell set");
        }
        if (bytes < off + 3 * ((size_t)h.n + (size_t)d.cells) * sizeof(double))
            fail(SLLG_E_ARG, "checkpoint truncated");
        const double* S = reinterpret_cast<const double*>(static_cast<const char*>(buf) + off);
        std::vector<double> v = normalised_spins(sys->n, S, false);
        clear_fault_copy(sys);
        std::vector<double> field(S + 3 * (size_t)h.n, S + 3 * ((size_t)h.n + (size_t)d.cells));
        if (sys->eng)
            sys->eng->set_spins(v);
        else
            sys->spins = v;
        if (sllg_set_rng(sys, h.seed, h.step) != SLLG_OK)
            fail(SLLG_E_DEVICE, sys->err);
        // the held field of the checkpoint (none: recomputed before the next step)
        sys->demag_valid = d.cells > 0;
        if (d.cells > 0) {
            if (sys->eng)
                sys->eng->demag_set(field);
            else
                sys->demag_pending = field;
        }
    });
}

namespace {

// Sites per tile of the two-launch step: a rebuild at the next run, state kept.
void set_tile_request(sllg_system* sys, int64_t value)
{
    if (value != sys->opt_tile_sites) {
        drop_engine(sys);
        sys->opt_tile_sites = value;
        sys->st.tile_request = (int)value;
    }
}

// The two-launch step also tries every tile size (a power of two from one
// workgroup's lanes to the largest the precision allows), each with its
// own launch shapes; the spins do not depend on the tiling, the m and E
// records only at FP64 rounding.
double autotune_with_tiles(sllg_system* s, int trial_steps, hipStream_t st)
{
    Engine& e0 = engine(s);
    if (fused_wanted(s) && e0.fused_capable())
        return autotune(s, trial_steps, st);
    const int64_t largest = s->prec == SLLG_FP64 ? tile_sites<double>() : tile_sites<float>();
    struct Best {
        double us = 1e30;
        int64_t tile = 0, remap = 1, scale = 100, graph = 0, order = 1, window = 1;
    } best;
    std::vector<int64_t> tiles;
    for (int64_t t = kBlockThreads; t <= largest; t *= 2)
        tiles.push_back(t);
    for (int64_t t : tiles) {
        set_tile_request(s, t);
        const double us = autotune(s, trial_steps, st);
        if (us < best.us)
            best = {us, t, s->opt_xcd_remap, s->opt_grid_scale_pct, s->opt_graph_steps, s->opt_tile_order,
                    s->opt_lds_window};
    }
    set_tile_request(s, best.tile);
    s->opt_xcd_remap = best.remap;
    s->opt_grid_scale_pct = best.scale;
    s->opt_graph_steps = best.graph;
    s->opt_tile_order = best.order;
    s->opt_lds_window = best.window;
    Engine& e = engine(s);
    e.set_remap((int)best.remap);
    e.set_grid_scale(best.scale / 100.0);
    e.set_tile_order((int)best.order, (int)s->opt_tile_group);
    e.set_window(best.window != 0);
    s->tuned = true;
    s->tuned_us = best.us;
    return best.us;
}

}  // namespace

sllg_status sllg_autotune(sllg_system* sys, int trial_steps, double* us_per_step, void* stream)
{
    return guard(sys, [&] {
        if (trial_steps < 2 || trial_steps > 100000)
            fail(SLLG_E_ARG, "trial_steps must be in 2..100000");
        const double us = autotune_with_tiles(sys, trial_steps, pick_stream(sys, stream));
        if (us_per_step)
            *us_per_step = us;
    });
}

sllg_status sllg_thermal_normals(int device, sllg_precision precision, uint64_t seed, uint64_t step,
                                 int64_t n, double* out)
{
    if (!out || n < 1 || n >= (int64_t(1) << kColBits) ||
        (precision != SLLG_FP32 && precision != SLLG_FP64))
        return SLLG_E_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return SLLG_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess)
        return SLLG_E_DEVICE;
    double* d = nullptr;
    if (hipMalloc(&d, 3 * (size_t)n * sizeof(double)) != hipSuccess)
        return SLLG_E_NOMEM;
    hipError_t e = precision == SLLG_FP32 ? launch_noise<float>(seed, step, (int)n, d, nullptr)
                                          : launch_noise<double>(seed, step, (int)n, d, nullptr);
    if (e == hipSuccess)
        e = hipMemcpy(out, d, 3 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e == hipSuccess ? SLLG_OK : SLLG_E_DEVICE;
}

sllg_status sllg_thermal_normals_noalloc(int device, sllg_precision precision, uint64_t seed, uint64_t step,
                                         int64_t n, double* out)
{
    if (!out || n < 1 || (precision != SLLG_FP32 && precision != SLLG_FP64)) {
        g_create_error = "out must not be NULL, n >= 1, precision SLLG_FP32 or SLLG_FP64";
        return SLLG_E_ARG;
    }
    if (n > kNoAllocMaxSites) {
        g_create_error = "n exceeds the no-allocation scratch (" + std::to_string(kNoAllocMaxSites) + " sites)";
        return SLLG_E_ARG;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return SLLG_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess)
        return SLLG_E_DEVICE;
    void* scratch = nullptr;
    size_t bytes = 0;
    if (noalloc_scratch(device, &scratch, &bytes) != hipSuccess || bytes < 3 * (size_t)n * sizeof(double)) {
        g_create_error = "no-allocation scratch unavailable on this device";
        return SLLG_E_DEVICE;
    }
    double* d = static_cast<double*>(scratch);
    hipError_t e = precision == SLLG_FP32 ? launch_noise<float>(seed, step, (int)n, d, nullptr)
                                          : launch_noise<double>(seed, step, (int)n, d, nullptr);
    if (e == hipSuccess)
        e = hipMemcpy(out, d, 3 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
    return e == hipSuccess ? SLLG_OK : SLLG_E_DEVICE;
}

sllg_status sllg_set_option(sllg_system* sys, const char* key, int64_t value)
{
    return guard(sys, [&] {
        if (!key)
            fail(SLLG_E_ARG, "key must not be NULL");
        const std::string k(key);
        if (k == "check_symmetry") {
            sys->opt_check_symmetry = value ? 1 : 0;
        } else if (k == "graph_steps") {
            if (value < -1 || value > 4096 || (value > 0 && (value & 1)))
                fail(SLLG_E_ARG, "graph_steps must be -1 (auto), 0, or even up to 4096");
            if (sys->eng && value > sys->eng->rec_cap())
                fail(SLLG_E_STATE, "graph_steps larger than the record buffer; set it before the first run");
            sys->opt_graph_steps = value;
        } else if (k == "grid_scale_pct") {
            if (value < 10 || value > 800)
                fail(SLLG_E_ARG, "grid_scale_pct must be in 10..800");
            sys->opt_grid_scale_pct = value;
            if (sys->eng)
                sys->eng->set_grid_scale(value / 100.0);
        } else if (k == "stencil") {
            sys->opt_stencil = value ? 1 : 0;   // applies to the next sllg_set_neighbours
        } else if (k == "mc_colouring") {
            if (value != 0 && value != 1)
                fail(SLLG_E_ARG, "mc_colouring must be 0 or 1");
            if (value != sys->opt_mc_colouring) {
                sys->opt_mc_colouring = value;
                if (sys->has_nb) {
                    HostStructure st = sys->st;
                    build_colours(st, value != 0);
                    drop_engine(sys);   // the colour lists are uploaded with the replica, state kept
                    sys->st = std::move(st);
                }
            }
        } else if (k == "tile_sites") {
            const int64_t largest = sys->prec == SLLG_FP64 ? tile_sites<double>() : tile_sites<float>();
            bool ok = value == 0;
            for (int64_t t = kBlockThreads; t <= largest && !ok; t *= 2)
                ok = value == t;
            if (!ok)
                fail(SLLG_E_ARG, "tile_sites must be 0 (automatic) or a power of two from " +
                                     std::to_string(kBlockThreads) + " to " + std::to_string(largest));
            set_tile_request(sys, value);   // rebuilt at the next run with the new tiling, state kept
        } else if (k == "lds_window") {
            if (value < 0 || value > 1)
                fail(SLLG_E_ARG, "lds_window must be 0 or 1");
            sys->opt_lds_window = value;
            if (sys->eng)
                sys->eng->set_window(value != 0);
        } else if (k == "tile_order") {
            if (value < 0 || value > 1)
                fail(SLLG_E_ARG, "tile_order must be 0 or 1");
            sys->opt_tile_order = value;
            if (sys->eng)
                sys->eng->set_tile_order((int)sys->opt_tile_order, (int)sys->opt_tile_group);
        } else if (k == "tile_group") {
            if (value < 0 || value > 4096)
                fail(SLLG_E_ARG, "tile_group must be in 0..4096");
            sys->opt_tile_group = value;
            if (sys->eng)
                sys->eng->set_tile_order((int)sys->opt_tile_order, (int)sys->opt_tile_group);
        } else if (k == "xcd_remap") {
            if (value < 0 || value > 2)
                fail(SLLG_E_ARG, "xcd_remap must be 0, 1 or 2");
            sys->opt_xcd_remap = value;
            if (sys->eng)
                sys->eng->set_remap((int)sys->opt_xcd_remap);
        } else if (k == "fused") {
            if (value < 0 || value > 2)
                fail(SLLG_E_ARG, "fused must be 0, 1 or 2");
            sys->opt_fused = value;
            if (sys->eng)
                sys->eng->set_fused(fused_wanted(sys));
        } else if (k == "fused_tile_x" || k == "fused_tile_y" || k == "fused_planes" || k == "fused_threads") {
            if (value < 0 || value > 0xFFFF)
                fail(SLLG_E_ARG, k + " must be in 0..65535");
            // fields not set yet start from the shape in use (once the engine exists)
            FusedShape f = sys->opt_fshape;
            const FusedShape cur = current_fused_shape(sys);
            if (f.px <= 0 && f.py <= 0 && f.planes <= 0 && f.bt <= 0)
                f = cur;
            if (k == "fused_tile_x")
                f.px = value > 0 ? (int)value + 2 : 0;
            else if (k == "fused_tile_y")
                f.py = value > 0 ? (int)value + 2 : 0;
            else if (k == "fused_planes")
                f.planes = (int)value;
            else
                f.bt = (int)value;
            if (value == 0) {
                sys->opt_fshape = FusedShape{};   // the model's shape at the next rebuild
            } else if (f.px > 0 && f.py > 0 && f.planes > 0 && f.bt > 0) {
                if (!fused_precision_ok(sys->st.lat, sys->n, sys->prec == SLLG_FP32 ? 4 : 8))
                    fail(SLLG_E_STATE, "no fused step: declare a lattice the fused step takes in this precision "
                                       "(sllg_set_lattice; FP64: simple cubic or bcc links)");
                // the device's LDS limit once it is open (MI355X: 160 KB per workgroup)
                if (!fused_shape_ok(f, sys->st.lat, sys->eng ? sys->eng->lds_limit() : (size_t)160 * 1024,
                                    sys->prec == SLLG_FP32 ? 4 : 8))
                    fail(SLLG_E_ARG, "fused shape out of range (tile " + std::to_string(f.px - 2) + " x " +
                                         std::to_string(f.py - 2) + ", " + std::to_string(f.planes) +
                                         " planes, " + std::to_string(f.bt) + " threads)");
                sys->opt_fshape = f;
                if (sys->eng && sys->eng->fused_capable())
                    sys->eng->set_fused_shape(f);
            } else {
                sys->opt_fshape = f;   // applied once every field is set
            }
        } else {
            fail(SLLG_E_ARG, "unknown option '" + k + "'");
        }
    });
}

sllg_status sllg_get_option(const sllg_system* sys, const char* key, int64_t* value)
{
    if (!sys || !key || !value)
        return SLLG_E_ARG;
    const std::string k(key);
    if (k == "check_symmetry")
        *value = sys->opt_check_symmetry;
    else if (k == "graph_steps")
        *value = graph_steps(sys);
    else if (k == "tile_sites") {
        HostStructure probe;
        probe.n = sys->n;
        probe.tile_request = (int)sys->opt_tile_sites;
        *value = tile_of(probe, sys->prec == SLLG_FP64 ? 8 : 4);
    }
    else if (k == "halo")
        *value = sys->has_nb ? sys->st.halo : -1;
    else if (k == "xcd_remap")
        *value = sys->opt_xcd_remap;
    else if (k == "tile_order")
        *value = sys->opt_tile_order;
    else if (k == "lds_window")
        *value = sys->opt_lds_window;
    else if (k == "tile_group")
        *value = sys->opt_tile_group;
    else if (k == "stencil")
        *value = sys->opt_stencil;
    else if (k == "mc_colouring")
        *value = sys->opt_mc_colouring;
    else if (k == "mc_colours")
        *value = sys->has_nb ? (int64_t)sys->st.colour_start.size() - 1 : -1;
    else if (k == "grid_scale_pct")
        *value = sys->opt_grid_scale_pct;
    else if (k == "tuned_ns_per_step")
        *value = sys->tuned ? (int64_t)(sys->tuned_us * 1e3) : -1;
    else if (k == "numeric_fault")
        *value = sys->eng ? (sys->eng->fault(nullptr) ? 1 : 0) : 0;   // waits for the queued work
    else if (k == "neighbour_format")
        *value = sys->has_nb ? (sys->st.stencil ? 1 : sys->st.wide ? 2 : 0) : -1;
    else if (k == "fused")
        *value = sys->opt_fused;
    else if (k == "lattice")
        *value = sys->st.lat.on ? (sys->st.lat.fusable ? 2 : 1) : 0;
    else if (k == "fused_active")
        *value = fused_will_run(sys) ? 1 : 0;
    else if (k == "fused_tile_x" || k == "fused_tile_y" || k == "fused_planes" || k == "fused_threads") {
        const FusedShape f = current_fused_shape(sys);
        *value = k == "fused_tile_x" ? f.px - 2 : k == "fused_tile_y" ? f.py - 2 : k == "fused_planes" ? f.planes : f.bt;
        if (f.px <= 0)
            *value = 0;
    } else
        return SLLG_E_ARG;
    return SLLG_OK;
}

}  // extern "C"
