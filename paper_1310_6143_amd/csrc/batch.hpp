// Batch engine: device buffers of every replica, the replica and work
// tables the kernels read, and the launch sequence of one chunk of Heun
// steps (optionally captured once as a HIP graph and replayed).
//
// A chunk of K steps is, for k = 0..K-1: predictor(k), corrector(k); then a
// measuring predictor pass and the record of the last step, the thermal
// average sums, and the advance of every replica's step counter and
// ping-pong parity.  Replicas that take fewer than K steps in a chunk exit
// the later launches at once, so one graph serves a changing batch.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "layout.hpp"
#include "prepare.hpp"

#ifndef SLLG_DEFAULT_REMAP
#define SLLG_DEFAULT_REMAP 1
#endif

namespace sllg {

inline void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        fail(e == hipErrorOutOfMemory ? SLLG_E_NOMEM : SLLG_E_DEVICE,
             std::string(what) + ": " + hipGetErrorString(e));
}

// Device memory source for replica buffers.
class Allocator {
public:
    virtual ~Allocator() = default;
    virtual void* alloc(size_t bytes) = 0;     // throws Failure on failure
    virtual void release(void* p) = 0;
};

class DirectAllocator final : public Allocator {
public:
    void* alloc(size_t bytes) override
    {
        void* p = nullptr;
        hip_check(hipMalloc(&p, std::max<size_t>(bytes, 256)), "hipMalloc");
        return p;
    }
    void release(void* p) override
    {
        if (p)
            (void)hipFree(p);
    }
};

// First-fit sub-allocator over one device allocation (the server's HBM
// budget), so admitting and retiring requests never calls hipMalloc/hipFree
// (hipFree would synchronise the device).
class PoolAllocator final : public Allocator {
public:
    explicit PoolAllocator(size_t bytes) : size_(round(bytes))
    {
        hip_check(hipMalloc(&base_, size_), "hipMalloc(pool)");
        free_[0] = size_;
    }
    ~PoolAllocator() override { (void)hipFree(base_); }
    void* alloc(size_t bytes) override
    {
        const size_t need = round(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > need)
                    free_[off + need] = len - need;
                used_[off] = need;
                in_use_ += need;
                return static_cast<char*>(base_) + off;
            }
        }
        fail(SLLG_E_BUDGET, "device pool exhausted");
    }
    void release(void* p) override
    {
        if (!p)
            return;
        const size_t off = static_cast<char*>(p) - static_cast<char*>(base_);
        auto it = used_.find(off);
        if (it == used_.end())
            return;
        size_t len = it->second;
        used_.erase(it);
        in_use_ -= len;
        size_t start = off;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + len) {
            len += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(off);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    size_t in_use() const { return in_use_; }
    size_t size() const { return size_; }
    static size_t round(size_t b) { return (b + 255) & ~size_t(255); }

private:
    void* base_ = nullptr;
    size_t size_ = 0;
    size_t in_use_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> used_;
};

inline size_t pad16(size_t b) { return (b + 15) & ~size_t(15); }

// Shape of the fused step's work items: thread region px x py (tile + 2 cells
// per axis), `planes` planes per item, bt threads per workgroup.
struct FusedShape {
    int px = 0, py = 0, planes = 0, bt = 0;
    bool operator==(const FusedShape& o) const
    {
        return px == o.px && py == o.py && planes == o.planes && bt == o.bt;
    }
};

constexpr int kFusedMinPlanes = 4;

// Most work items any allowed shape gives (smallest tiles, fewest planes).
inline int64_t fused_item_cap(const HostLattice& L)
{
    const int64_t t = kFusedMinEdge - 2, p = std::max(std::min(kFusedMinPlanes, L.nz), 1);
    return ((L.nx + t - 1) / t) * ((L.ny + t - 1) / t) * ((L.nz + p - 1) / p);
}

// LDS bytes of one plane of the fused kernel (the tile, the ring and one
// more ring; fused_plane_bytes of kernels.hpp).
inline int fused_plane_bytes(const FusedShape& f, int nb, size_t real_bytes)
{
    return fused_plane_bytes(f.px, f.py, nb, real_bytes, f.bt);
}

// A shape the kernels take for lattice L in a precision (bytes per real):
// the region fits the block (and, in FP64, the LDS row), the LDS planes fit
// the device (lds_limit bytes per workgroup) and each wave copies at most
// fused_chunks_per_wave chunks per plane; items have at least
// kFusedMinPlanes planes (all of them on thinner lattices).
inline bool fused_shape_ok(const FusedShape& f, const HostLattice& L, size_t lds_limit, size_t real_bytes)
{
    if (!fused_block_ok(L.kind, f.bt, real_bytes) || f.px < kFusedMinEdge || f.py < kFusedMinEdge ||
        f.px > 0x7FFF || f.py > 0x7FFF || (int64_t)f.px * f.py > f.bt || f.planes < std::min(kFusedMinPlanes, L.nz))
        return false;
    if (real_bytes == 8 && f.px + 2 > fused_row_slots(real_bytes, f.bt))
        return false;
    if ((int64_t)f.py > 0x7FFF / (L.nb * 64) ||
        fused_plane_chunks(f.px, f.py, L.nb, real_bytes, f.bt) > fused_chunks_per_wave(real_bytes) * (f.bt / 64))
        return false;
    return fused_lds_bytes(L.kind, fused_plane_bytes(f, L.nb, real_bytes), f.bt) + fused_static_lds(f.bt, real_bytes) <=
           lds_limit;
}

// Work items of a lattice for a shape.
inline int64_t fused_items(const HostLattice& L, const FusedShape& f)
{
    const int64_t tx = f.px - 2, ty = f.py - 2;
    return ((L.nx + tx - 1) / tx) * ((L.ny + ty - 1) / ty) * ((L.nz + f.planes - 1) / f.planes);
}

// Candidate shapes for a lattice (the autotuner times them; the first is
// the model's choice).  resident(f) gives the workgroups the device holds
// at once for shape f.  FP32: the planes per item are chosen so that the
// items fill whole rounds of the resident workgroups; the model counts
// wave-instructions of one item (predictor on planes + 2 on every wave,
// corrector on planes on the waves that hold tile cells, plane copies on
// planes + 4) times rounds.  FP64 (the predictor's FP64 noise dominates,
// and a partly idle last round costs little): an item's predictor planes
// plus a fifth of its corrector planes (per wave) times the items per
// resident workgroup, at least one.
template <typename Resident>
inline std::vector<FusedShape> fused_candidates(const HostLattice& L, size_t lds_limit, size_t real_bytes,
                                                Resident&& resident, int max_count)
{
    struct Scored {
        double cost;
        FusedShape f;
    };
    std::vector<Scored> all;
    for (int bt : {256, 512, 1024}) {
        for (int px = kFusedMinEdge; px <= 64; ++px)
            for (int py = kFusedMinEdge; py <= bt / kFusedMinEdge; ++py) {
                FusedShape f{px, py, std::min(kFusedMinPlanes, L.nz), bt};
                if (!fused_shape_ok(f, L, lds_limit, real_bytes))
                    continue;
                const int tx = px - 2, ty = py - 2;
                if (tx > L.nx + 6 || ty > L.ny + 6)   // far wider than the lattice
                    continue;
                // FP64: of the tiles that give the same number of columns,
                // only the smallest (the least ring work)
                if (real_bytes == 8 && ((tx > kFusedMinEdge - 2 && (L.nx + tx - 2) / (tx - 1) == (L.nx + tx - 1) / tx) ||
                                        (ty > kFusedMinEdge - 2 && (L.ny + ty - 2) / (ty - 1) == (L.ny + ty - 1) / ty)))
                    continue;
                const int R = std::max(resident(f), 1);
                const int64_t cols = (int64_t)((L.nx + tx - 1) / tx) * ((L.ny + ty - 1) / ty);
                // predictor phases on every wave; the corrector phases only
                // on waves that hold tile cells (the tile's threads come first)
                const int waves = (px * py + 63) / 64, tile_waves = (tx * ty + 63) / 64;
                for (int segs = 1; segs <= L.nz; ++segs) {
                    const int planes = (L.nz + segs - 1) / segs;
                    if (planes < std::min(kFusedMinPlanes, L.nz))
                        break;
                    if (segs > 1 && (L.nz + segs - 2) / (segs - 1) == planes)
                        continue;   // the same planes as fewer segments
                    const int64_t items = cols * ((L.nz + planes - 1) / planes);
                    f.planes = planes;
                    if (real_bytes == 8) {
                        const double item = (planes + 2) + (double)tile_waves / waves * planes * 0.2;
                        all.push_back({std::max((double)items / R, 1.0) * item, f});
                        continue;
                    }
                    const double item = waves * ((planes + 2) * 1.0 + (planes + 4) * 0.25) + tile_waves * planes * 0.4;
                    const double rounds = std::ceil((double)items / R);
                    all.push_back({rounds * item * R, f});
                }
            }
    }
    std::sort(all.begin(), all.end(), [](const Scored& a, const Scored& b) { return a.cost < b.cost; });
    std::vector<FusedShape> out;
    for (const auto& a : all) {
        if ((int)out.size() >= max_count)
            break;
        bool dup = false;
        for (const auto& o : out)
            dup = dup || o == a.f;
        if (!dup)
            out.push_back(a.f);
    }
    return out;
}

// Bytes of device memory one replica needs (used for admission).
inline size_t replica_bytes(const HostStructure& s, const HostMaterials& m, size_t real_bytes,
                            int64_t rec_cap, int avg_cap)
{
    auto r = [](size_t b) { return PoolAllocator::round(b); };
    const size_t n = (size_t)s.n;
    const size_t tile = (size_t)tile_of(s, real_bytes);
    const size_t blocks = (n + tile - 1) / tile;
    size_t b = 3 * r(spin_buffer_bytes(s.n, real_bytes) + 16) + r(4);  // S[2], Sp, the fault flag
    if (s.stencil)
        b += r(pad16(n)) + r(s.pat_tab.size() * 4) + r(s.pat_start.size() * 2) + r(s.pat_far.size() * 2);
    else if (s.wide)
        b += r(2 * n) + r(s.w_tab.size() * 4) + r(s.w_near.size() * 2);
    else
        b += r(s.nb.size() * 4) + r(s.slice_off.size() * 8) + r(4 * n);
    if (!s.colour_sites.empty())
        b += r(4 * n) + ((s.stencil || s.wide) ? r(2 * n) : 0);
    if (m.per_site_material)
        b += r(n);
    if (m.per_site_axis)
        b += r(3 * n * real_bytes);
    if (s.demag.on) {
        const size_t nc = (size_t)s.demag.cells;
        b += 2 * r(4 * n) + r(4 * (nc + 1)) + 3 * r(3 * nc * real_bytes) + r(nc * real_bytes) +
             r(3 * nc * (size_t)demag_chunks(s.demag.cells) * real_bytes);
    }
    if (s.lat.on && s.lat.fusable && real_bytes == 4) {
        size_t ent = 0;
        for (const auto& p : s.lat.pats)
            ent += p.size();
        b += r(ent * sizeof(FusedEntry)) + r(s.lat.pats.size() * 16) + r(s.lat.plane_pat.size()) +
             r((size_t)fused_item_cap(s.lat) * 64);
    }
    b += r(m.mat_mu.size() * sizeof(MaterialDev<double>));
    const size_t groups = (blocks + kGroupTiles - 1) / kGroupTiles;
    b += r(groups * 32);
    b += r(blocks * 32) + r((size_t)std::max<int64_t>(rec_cap, 1) * 32) +
         r((size_t)std::max(avg_cap, 1) * 40);
    return b;
}

// Plane stride of a stencil lattice in tiles: the median over sites of
// |column - row| of the far links (those beyond the LDS halo), divided by
// the tile size; 0 when there are none or they are within two tiles.
inline int plane_tiles(const HostStructure& s, int tile)
{
    if (!s.stencil)
        return 0;
    const int np = (int)s.pat_start.size() - 1;
    std::vector<int64_t> uses(np, 0);
    for (uint8_t p : s.pat_id)
        ++uses[p];
    std::vector<std::pair<int64_t, int64_t>> far;   // (|offset|, sites)
    int64_t total = 0;
    for (int p = 0; p < np; ++p)
        for (int k = s.pat_far[p]; k < s.pat_start[p + 1]; ++k) {
            far.emplace_back(std::llabs((int64_t)(s.pat_tab[k] >> 4)), uses[p]);
            total += uses[p];
        }
    if (total == 0)
        return 0;
    std::sort(far.begin(), far.end());
    int64_t acc = 0, median = 0;
    for (const auto& f : far)
        if ((acc += f.second) * 2 >= total) {
            median = f.first;
            break;
        }
    const int64_t pt = (median + tile / 2) / tile;
    return pt >= 2 && pt < (int64_t(1) << 30) ? (int)pt : 0;
}

// Order in which a replica's tiles are listed for the step launches.  With
// a plane stride of pt tiles, groups of `group` adjacent tile columns are
// swept plane after plane, so a tile's far neighbours (one plane away) were
// read a few tiles earlier and are still in the L2.
inline std::vector<int32_t> tile_order(int blocks, int pt, int group)
{
    std::vector<int32_t> o;
    o.reserve((size_t)blocks);
    if (pt < 2 || group <= 0 || pt >= blocks) {
        for (int b = 0; b < blocks; ++b)
            o.push_back(b);
        return o;
    }
    const int64_t nz = ((int64_t)blocks + pt - 1) / pt;
    for (int c0 = 0; c0 < pt; c0 += group)
        for (int64_t z = 0; z < nz; ++z)
            for (int c = c0; c < std::min(c0 + group, pt); ++c) {
                const int64_t t = z * pt + c;
                if (t < blocks)
                    o.push_back((int32_t)t);
            }
    return o;
}

template <typename R>
class Batch {
public:
    struct Slot {
        bool used = false;
        ReplicaDev<R> rec{};
        std::vector<void*> mem;
        int64_t rec_cap = 0;
        int avg_cap = 0;
        size_t bytes = 0;
        int plane_tiles = 0;     // see plane_tiles()
        int32_t* d_colour = nullptr;            // Monte Carlo: sites by colour class
        uint16_t* d_colour_pid = nullptr;       // their stencil patterns, in the same order (stencil forms)
        std::vector<int64_t> colour_start;      // [n_colours + 1]
        // fused step (kFused): patterns, shape and work items
        HostLattice lat;
        FusedShape fshape;
        int64_t f_cap_items = 0;                // items the partials buffer holds
        std::vector<FusedItem> f_items;
    };

    Batch(int device, Allocator* alloc, int max_replicas)
        : device_(device), alloc_(alloc), slots_(max_replicas)
    {
        hip_check(hipSetDevice(device_), "hipSetDevice");
        hip_check(hipMalloc(&d_reps_, sizeof(ReplicaDev<R>) * (size_t)max_replicas), "hipMalloc(reps)");
        hip_check(hipMalloc(&d_nwork_, sizeof(int)), "hipMalloc(nwork)");
        hip_check(hipMemset(d_nwork_, 0, sizeof(int)), "hipMemset");
        host_reps_.resize(max_replicas);
        // pinned staging of the replica table: its per-chunk upload is then a
        // plain DMA on the work stream
        hip_check(hipHostMalloc((void**)&pinned_reps_, sizeof(ReplicaDev<R>) * (size_t)max_replicas),
                  "hipHostMalloc(reps)");
        for (int v = 0; v < 3; ++v) {
            int& res = resident_v_[v];
            res = resident_blocks<R>(device_, v);
            if (res < 8)
                res = 8 * 256;
            res &= ~7;
        }
        resident_ = resident_v_[0];
        // A group's tiles stream about 9 sizeof(R) bytes per site through the
        // L2 per launch (the corrector reads S' and S and writes S); the
        // plane-to-plane reuse spans two planes of a group, kept within a
        // quarter of one L2 (the L2 of one XCD on MI355X): group_sites_ is
        // that budget in sites.
        int l2 = 0;
        if (hipDeviceGetAttribute(&l2, hipDeviceAttributeL2CacheSize, device_) != hipSuccess || l2 <= 0)
            l2 = 4 << 20;
        group_sites_ = (int64_t)l2 / (4 * 9 * (int64_t)sizeof(R));
    }

    ~Batch()
    {
        (void)hipSetDevice(device_);
        drop_graph();
        for (size_t q = 0; q < slots_.size(); ++q)
            if (slots_[q].used)
                remove(q);
        (void)hipFree(d_reps_);
        (void)hipFree(d_work_);
        (void)hipFree(d_fwork_);
        (void)hipFree(d_nwork_);
        (void)hipFree(d_torque_work_);
        (void)hipFree(d_torque_);
        (void)hipHostFree(pinned_reps_);
    }

    Batch(const Batch&) = delete;
    Batch& operator=(const Batch&) = delete;

    // Wait for every launch this batch queued.  Host-side changes of the
    // device tables and buffers go through synchronous copies, which are not
    // ordered with the (non-blocking) work stream, so they wait first.
    void quiesce()
    {
        if (last_stream_) {
            hip_check(hipStreamSynchronize(last_stream_), "hipStreamSynchronize");
            last_stream_ = nullptr;
        }
    }

    int capacity() const { return (int)slots_.size(); }
    Slot& slot(int q) { return slots_[q]; }
    ReplicaDev<R>& mirror(int q) { return slots_[q].rec; }
    // The replica set, shapes or launch options changed: the work lists are
    // rebuilt at the next launch, and the replica table uploaded.
    void mark_dirty()
    {
        dirty_ = true;
        lists_dirty_ = true;
    }
    // Only scalar fields of the replica table changed (step counts, record
    // flags): the next launch uploads the table and keeps the lists, unless
    // the set of replicas that run changed.
    void mark_scalars_dirty() { dirty_ = true; }

    // Allocate and fill the buffers of a new replica; returns its slot.
    int add(const HostStructure& s, const HostMaterials& m, const Dynamics& d,
            const std::vector<double>& S0, int64_t rec_cap, int avg_cap)
    {
        quiesce();
        int q = -1;
        for (size_t i = 0; i < slots_.size(); ++i)
            if (!slots_[i].used) {
                q = (int)i;
                break;
            }
        if (q < 0)
            fail(SLLG_E_BUDGET, "no free replica slot");
        Slot& sl = slots_[q];
        sl = Slot{};
        sl.rec_cap = std::max<int64_t>(rec_cap, 1);
        sl.avg_cap = std::max(avg_cap, 1);
        const size_t n = (size_t)s.n;
        const size_t tile = (size_t)tile_of(s, sizeof(R));
        const size_t blocks = (n + tile - 1) / tile;
        try {
            auto get = [&](size_t bytes) {
                void* p = alloc_->alloc(bytes);
                sl.mem.push_back(p);
                return p;
            };
            ReplicaDev<R>& r = sl.rec;
            const size_t sb = spin_buffer_bytes(s.n, sizeof(R));
            // 16 bytes past the last site: the fused step copies 16 bytes per site
            r.S[0] = (R*)get(sb + 16);
            r.S[1] = (R*)get(sb + 16);
            r.Sp = (R*)get(sb);
            r.fault = (int32_t*)get(4);
            hip_check(hipMemset(r.fault, 0, 4), "clear fault flag");
            // the padding is staged with the last tile's window: keep it finite
            for (void* p : {(void*)r.S[0], (void*)r.S[1]})
                hip_check(hipMemset(p, 0, sb + 16), "clear spins");
            hip_check(hipMemset(r.Sp, 0, sb), "clear spins");
            r.nb = nullptr;
            r.slice_off = nullptr;
            r.deg = nullptr;
            r.pat_id = nullptr;
            r.pat_tab = nullptr;
            r.pat_start = nullptr;
            r.pat_far = nullptr;
            r.w_pid = nullptr;
            r.w_tab = nullptr;
            r.w_near = nullptr;
            if (s.wide) {
                uint16_t* pid = (uint16_t*)get(2 * n);
                int32_t* tab = (int32_t*)get(s.w_tab.size() * 4);
                uint16_t* nn = (uint16_t*)get(s.w_near.size() * 2);
                hip_check(hipMemcpy(pid, s.w_pid.data(), 2 * n, hipMemcpyHostToDevice), "upload pattern ids");
                hip_check(hipMemcpy(tab, s.w_tab.data(), s.w_tab.size() * 4, hipMemcpyHostToDevice), "upload patterns");
                hip_check(hipMemcpy(nn, s.w_near.data(), s.w_near.size() * 2, hipMemcpyHostToDevice),
                          "upload pattern splits");
                r.w_pid = pid;
                r.w_tab = tab;
                r.w_near = nn;
            } else if (s.stencil) {
                uint8_t* pid = (uint8_t*)get(pad16(n));
                int32_t* tab = (int32_t*)get(std::max<size_t>(s.pat_tab.size(), 1) * 4);
                uint16_t* ps = (uint16_t*)get(s.pat_start.size() * 2);
                uint16_t* pf = (uint16_t*)get(std::max<size_t>(s.pat_far.size(), 1) * 2);
                hip_check(hipMemset(pid, 0, pad16(n)), "clear pattern ids");
                hip_check(hipMemcpy(pid, s.pat_id.data(), n, hipMemcpyHostToDevice), "upload pattern ids");
                hip_check(hipMemcpy(pf, s.pat_far.data(), s.pat_far.size() * 2, hipMemcpyHostToDevice),
                          "upload pattern splits");
                hip_check(hipMemcpy(tab, s.pat_tab.data(), s.pat_tab.size() * 4, hipMemcpyHostToDevice),
                          "upload patterns");
                hip_check(hipMemcpy(ps, s.pat_start.data(), s.pat_start.size() * 2, hipMemcpyHostToDevice),
                          "upload pattern starts");
                r.pat_id = pid;
                r.pat_tab = tab;
                r.pat_start = ps;
                r.pat_far = pf;
            } else {
                uint32_t* nb = (uint32_t*)get(std::max<size_t>(s.nb.size(), 1) * 4);
                int64_t* so = (int64_t*)get(s.slice_off.size() * 8);
                uint32_t* dg = (uint32_t*)get(4 * n);
                hip_check(hipMemcpy(nb, s.nb.data(), s.nb.size() * 4, hipMemcpyHostToDevice), "upload nb");
                hip_check(hipMemcpy(so, s.slice_off.data(), s.slice_off.size() * 8, hipMemcpyHostToDevice),
                          "upload slices");
                hip_check(hipMemcpy(dg, s.deg.data(), 4 * n, hipMemcpyHostToDevice), "upload deg");
                r.nb = nb;
                r.slice_off = so;
                r.deg = dg;
            }
            r.matid = nullptr;
            r.axis = nullptr;
            if (m.per_site_material) {
                uint8_t* mi = (uint8_t*)get(n);
                hip_check(hipMemcpy(mi, m.matid.data(), n, hipMemcpyHostToDevice), "upload matid");
                r.matid = mi;
            }
            if (m.per_site_axis) {
                std::vector<R> ax(3 * n);
                for (size_t i = 0; i < 3 * n; ++i)
                    ax[i] = (R)m.axis_site[i];
                R* a = (R*)get(3 * n * sizeof(R));
                hip_check(hipMemcpy(a, ax.data(), 3 * n * sizeof(R), hipMemcpyHostToDevice), "upload axes");
                r.axis = a;
            }
            r.dm_cell = r.dm_start = r.dm_atoms = nullptr;
            r.dm_pos = r.dm_self = nullptr;
            r.dm_m = r.dm_field = r.dm_part = nullptr;
            if (s.demag.on) {
                const HostDemag& dm = s.demag;
                const size_t nc = (size_t)dm.cells;
                std::vector<double> centre, self;
                demag_cells(dm, m, centre, self);
                std::vector<R> cR(centre.begin(), centre.end()), sR(self.begin(), self.end());
                int32_t* dc = (int32_t*)get(4 * n);
                int32_t* ds = (int32_t*)get(4 * (nc + 1));
                int32_t* da = (int32_t*)get(4 * n);
                R* dp = (R*)get(3 * nc * sizeof(R));
                R* dsf = (R*)get(nc * sizeof(R));
                R* dmm = (R*)get(3 * nc * sizeof(R));
                R* df = (R*)get(3 * nc * sizeof(R));
                const int chunks = demag_chunks(dm.cells);
                R* dpart = (R*)get(3 * nc * (size_t)chunks * sizeof(R));
                hip_check(hipMemcpy(dc, dm.cell_of.data(), 4 * n, hipMemcpyHostToDevice), "upload macrocells");
                hip_check(hipMemcpy(ds, dm.start.data(), 4 * (nc + 1), hipMemcpyHostToDevice), "upload macrocells");
                hip_check(hipMemcpy(da, dm.atoms.data(), 4 * n, hipMemcpyHostToDevice), "upload macrocells");
                hip_check(hipMemcpy(dp, cR.data(), 3 * nc * sizeof(R), hipMemcpyHostToDevice), "upload macrocells");
                hip_check(hipMemcpy(dsf, sR.data(), nc * sizeof(R), hipMemcpyHostToDevice), "upload macrocells");
                hip_check(hipMemset(dmm, 0, 3 * nc * sizeof(R)), "clear macrocells");
                hip_check(hipMemset(df, 0, 3 * nc * sizeof(R)), "clear macrocells");
                r.dm_cell = dc;
                r.dm_start = ds;
                r.dm_atoms = da;
                r.dm_pos = dp;
                r.dm_self = dsf;
                r.dm_m = dmm;
                r.dm_field = df;
                r.dm_part = dpart;
            }
            r.f_ent = nullptr;
            r.f_pat = nullptr;
            r.f_plane = nullptr;
            r.f_partials = nullptr;
            r.f_px = r.f_py = r.f_items = 0;
            if (fused_precision_ok(s.lat, s.n, sizeof(R))) {
                size_t ent = 0;
                for (const auto& p : s.lat.pats)
                    ent += p.size();
                sl.lat = s.lat;
                sl.f_cap_items = fused_item_cap(s.lat);
                r.f_ent = get(std::max<size_t>(ent, 1) * sizeof(FusedEntry));
                r.f_pat = (const int32_t*)get(s.lat.pats.size() * 16);
                if (!s.lat.plane_pat.empty()) {
                    uint8_t* pp = (uint8_t*)get(s.lat.plane_pat.size());
                    hip_check(hipMemcpy(pp, s.lat.plane_pat.data(), s.lat.plane_pat.size(), hipMemcpyHostToDevice),
                              "upload plane patterns");
                    r.f_plane = pp;
                }
                r.f_partials = (double*)get((size_t)sl.f_cap_items * 2 * 4 * sizeof(double));
            }
            r.mat = (MaterialDev<R>*)get(m.mat_mu.size() * sizeof(MaterialDev<R>));
            r.partials = (double*)get(blocks * 4 * sizeof(double));
            const size_t groups = (blocks + kGroupTiles - 1) / kGroupTiles;
            r.group_partials = (double*)get(groups * 4 * sizeof(double));
            r.records = (double*)get((size_t)sl.rec_cap * 4 * sizeof(double));
            r.acc = (double*)get((size_t)sl.avg_cap * 5 * sizeof(double));
            r.flags = 0;
            fill_parameters(r, s, m, d);
            if (r.f_partials)
                sl.fshape = fused_candidates(sl.lat, lds_limit(), sizeof(R),
                                             [&](const FusedShape& f) { return fused_resident(sl.lat, f); }, 1)
                                .at(0);
            upload_materials(q, m, d);
            r.parity = 0;
            r.nsteps = 0;
            r.rec_pos = 0;
            r.avg_first = 0;
            r.avg_block_len = 1;
            r.avg_blocks = 0;
            set_spins(q, S0);
            sl.bytes = replica_bytes(s, m, sizeof(R), sl.rec_cap, sl.avg_cap);
            sl.plane_tiles = plane_tiles(s, (int)tile);
            if (!s.colour_sites.empty()) {
                sl.d_colour = (int32_t*)get(4 * n);
                if (s.stencil || s.wide) {
                    // each trial's pattern, read beside its site instead of after it
                    std::vector<uint16_t> pid(n);
                    for (size_t k = 0; k < n; ++k) {
                        const size_t i = (size_t)s.colour_sites[k];
                        pid[k] = s.stencil ? (uint16_t)s.pat_id[i] : s.w_pid[i];
                    }
                    sl.d_colour_pid = (uint16_t*)get(2 * n);
                    hip_check(hipMemcpy(sl.d_colour_pid, pid.data(), 2 * n, hipMemcpyHostToDevice),
                              "upload colour-class patterns");
                }
                hip_check(hipMemcpy(sl.d_colour, s.colour_sites.data(), 4 * n, hipMemcpyHostToDevice),
                          "upload colour classes");
                sl.colour_start = s.colour_start;
            }
            sl.used = true;
        } catch (...) {
            for (void* p : sl.mem)
                alloc_->release(p);
            sl = Slot{};
            throw;
        }
        mark_dirty();
        return q;
    }

    void remove(int q)
    {
        Slot& sl = slots_[q];
        if (!sl.used)
            return;
        quiesce();
        for (void* p : sl.mem)
            alloc_->release(p);
        sl = Slot{};
        mark_dirty();
    }

    void upload_materials(int q, const HostMaterials& m, const Dynamics& d)
    {
        const auto table = material_table<R>(m, d);
        quiesce();
        hip_check(hipMemcpy((void*)slots_[q].rec.mat, table.data(), table.size() * sizeof(MaterialDev<R>),
                            hipMemcpyHostToDevice),
                  "upload materials");
        upload_fused(q);
    }

    // Fused step: pattern entries for the slot's shape (LDS offsets depend
    // on the region width; J / mu_ref from the replica's table) and its work
    // items.
    void upload_fused(int q)
    {
        Slot& sl = slots_[q];
        ReplicaDev<R>& r = sl.rec;
        if (!r.f_partials)
            return;
        const FusedShape f = sl.fshape;
        const HostLattice& L = sl.lat;
        // LDS planes hold slots basis-major: (b, row, column) -> b * area + row * SW + column
        const int SW = f.px + 2, area = (f.px + 2) * (f.py + 2);
        std::vector<int32_t> hdr;
        std::vector<FusedEntry> ent;
        for (size_t p = 0; p < L.pats.size(); ++p) {
            const int b = L.pat_b[p];
            int cnt[3] = {0, 0, 0};
            hdr.push_back((int32_t)ent.size());
            for (const FusedLink& l : L.pats[p]) {
                ++cnt[l.dz + 1];
                const int slot_off = ((int)l.bp - b) * area + l.dy * SW + l.dx;
                ent.push_back(FusedEntry{slot_off * 16, (float)r.jt[l.type]});
            }
            hdr.push_back(cnt[0]);
            hdr.push_back(cnt[1]);
            hdr.push_back(cnt[2]);
        }
        quiesce();
        if (!ent.empty())
            hip_check(hipMemcpy((void*)r.f_ent, ent.data(), ent.size() * sizeof(FusedEntry), hipMemcpyHostToDevice),
                      "upload fused entries");
        hip_check(hipMemcpy((void*)r.f_pat, hdr.data(), hdr.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                  "upload fused patterns");
        r.f_px = f.px;
        r.f_py = f.py;
        sl.f_items.clear();
        const int tx = f.px - 2, ty = f.py - 2;
        int32_t idx = 0;
        for (int z0 = 0; z0 < L.nz; z0 += f.planes)
            for (int y0 = 0; y0 < L.ny; y0 += ty)
                for (int x0 = 0; x0 < L.nx; x0 += tx)
                    sl.f_items.push_back(FusedItem{q, x0, y0, z0, std::min(z0 + f.planes, L.nz), idx++});
        if ((int64_t)sl.f_items.size() > sl.f_cap_items)
            fail(SLLG_E_STATE, "fused work items exceed their buffer");
        r.f_items = idx;
        mark_dirty();
    }

    // Shape of replica q's fused step (fused_shape_ok).
    void set_fused_shape(int q, const FusedShape& f)
    {
        Slot& sl = slots_[q];
        if (!sl.rec.f_partials)
            fail(SLLG_E_STATE, "the replica has no fused step");
        if (!fused_shape_ok(f, sl.lat, lds_limit(), sizeof(R)))
            fail(SLLG_E_ARG, "fused shape out of range");
        if (sl.fshape == f)
            return;
        sl.fshape = f;
        upload_fused(q);
        drop_graph();
    }
    FusedShape fused_shape(int q) const { return slots_[q].fshape; }
    const HostLattice& lattice(int q) const { return slots_[q].lat; }
    bool fused_active() const { return fused_mode_; }
    void set_fused(bool on)
    {
        if (on != fused_on_) {
            fused_on_ = on;
            mark_dirty();
        }
    }
    // Workgroups of the fused kernel the device holds at once for lattice L
    // in shape f: the register limit (queried once per kernel) and the LDS
    // of the compute units.
    int fused_resident(const HostLattice& L, const FusedShape& f)
    {
        const int key = ((L.kind * 4 + L.nb) * 4) + (f.bt >> 8);
        auto it = fused_occ_.find(key);
        if (it == fused_occ_.end())
            it = fused_occ_.emplace(key, fused_resident_blocks<R>(device_, L.kind, L.nb, f.bt, 16)).first;
        int cus = 0, lds_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device_) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device_) != hipSuccess ||
            lds_cu <= 0)
            lds_cu = 160 * 1024;
        const size_t per_wg =
            fused_lds_bytes(L.kind, fused_plane_bytes(f, L.nb, sizeof(R)), f.bt) + fused_static_lds(f.bt, sizeof(R));
        const int by_lds = (int)std::max<size_t>(1, (size_t)lds_cu / per_wg);
        const int by_regs = std::max(1, it->second / cus);
        return cus * std::min(by_lds, by_regs);
    }
    size_t lds_limit()
    {
        if (lds_limit_ == 0)
            lds_limit_ = fused_lds_limit(device_);
        return lds_limit_;
    }
    std::vector<FusedShape> fused_candidate_shapes(int q, int max_count)
    {
        const HostLattice& L = slots_[q].lat;
        return fused_candidates(L, lds_limit(), sizeof(R), [&](const FusedShape& f) { return fused_resident(L, f); },
                                max_count);
    }

    // Write the current state (spins are normalised doubles, 3n).
    void set_spins(int q, const std::vector<double>& S)
    {
        ReplicaDev<R>& r = slots_[q].rec;
        quiesce();
        std::vector<R> tmp(S.size());
        for (size_t i = 0; i < S.size(); ++i)
            tmp[i] = (R)S[i];
        hip_check(hipMemcpy(r.S[r.parity], tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice),
                  "upload spins");
        hip_check(hipMemset(r.fault, 0, 4), "clear fault flag");   // new state, no fault
    }

    // Non-finite-spin flag of replica q (set by the step and Monte Carlo
    // kernels).  fault(): waits for stream st and reads it; fault_async():
    // queues a copy of it into host (pinned memory) on st.
    bool fault(int q, hipStream_t st)
    {
        int32_t v = 0;
        quiesce();   // the last stream the batch ran on
        if (st)
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        hip_check(hipMemcpy(&v, slots_[q].rec.fault, 4, hipMemcpyDeviceToHost), "read fault flag");
        return v != 0;
    }
    void fault_async(int q, int32_t* host, hipStream_t st)
    {
        hip_check(hipMemcpyAsync(host, slots_[q].rec.fault, 4, hipMemcpyDeviceToHost, st), "queue fault flag copy");
    }

    void get_spins(int q, double* out, hipStream_t st)
    {
        ReplicaDev<R>& r = slots_[q].rec;
        std::vector<R> tmp(3 * (size_t)r.n);
        quiesce();
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        hip_check(hipMemcpy(tmp.data(), r.S[r.parity], tmp.size() * sizeof(R), hipMemcpyDeviceToHost),
                  "download spins");
        for (size_t i = 0; i < tmp.size(); ++i)
            out[i] = (double)tmp[i];
    }

    // Upload the replica records and the work list when something changed.
    // Bring the device tables up to date before a launch.  With a stream,
    // the replica table goes up as an asynchronous copy on it (from pinned
    // memory, which the next call reuses only after quiesce()).
    void sync_tables(hipStream_t st = nullptr)
    {
        if (!dirty_)
            return;
        quiesce();
        // A replica's flags must match the buffers it owns: the kernels pick
        // the neighbour layout, material and axis lookups from the flags.
        for (const auto& sl : slots_) {
            if (!sl.used)
                continue;
            const ReplicaDev<R>& r = sl.rec;
            const bool stencil = (r.flags & kStencil) != 0, wide = (r.flags & kWide) != 0;
            if ((stencil && wide) || (stencil && (!r.pat_id || !r.pat_tab || !r.pat_start || !r.pat_far)) ||
                (wide && (!r.w_pid || !r.w_tab || !r.w_near || r.w_len <= 0 || r.n_patterns <= 0)) ||
                (!stencil && !wide && (!r.nb || !r.slice_off || !r.deg)) ||
                ((r.flags & kPerSiteMaterial) && !r.matid) || ((r.flags & kPerSiteAxis) && !r.axis) ||
                ((r.flags & kAverage) && (!(r.flags & kRecord) || !r.acc)))
                fail(SLLG_E_STATE, "replica flags do not match its buffers");
        }
        for (size_t q = 0; q < slots_.size(); ++q) {
            host_reps_[q] = slots_[q].used ? slots_[q].rec : ReplicaDev<R>{};
            if (slots_[q].used && !window_)
                host_reps_[q].flags |= kDirect;
            if (!slots_[q].used)
                host_reps_[q].nsteps = 0;
        }
        // the work lists hold the replicas that run: rebuilt when that set changed
        std::vector<char> active(slots_.size());
        for (size_t q = 0; q < slots_.size(); ++q)
            active[q] = slots_[q].used && slots_[q].rec.nsteps > 0;
        if (active != active_)
            lists_dirty_ = true;
        if (lists_dirty_)
            build_lists();
        active_ = active;
        lists_dirty_ = false;
        // whether the fused step launches need the record code (the record
        // flags change without the lists); a captured chunk holds the
        // kernel variant chosen here
        bool any_rec = false;
        for (const auto& sl : slots_)
            if (sl.used && sl.rec.nsteps > 0 && (sl.rec.flags & kRecord))
                any_rec = true;
        if (any_rec != fused_rec_)
            drop_graph();
        fused_rec_ = any_rec;
        const size_t bytes = sizeof(ReplicaDev<R>) * host_reps_.size();
        if (st) {
            std::memcpy(pinned_reps_, host_reps_.data(), bytes);
            hip_check(hipMemcpyAsync(d_reps_, pinned_reps_, bytes, hipMemcpyHostToDevice, st), "upload replicas");
            last_stream_ = st;
        } else {
            hip_check(hipMemcpy(d_reps_, host_reps_.data(), bytes, hipMemcpyHostToDevice), "upload replicas");
        }
        dirty_ = false;
    }

    // The launch variant, the two-launch work list and the fused item list of
    // the replicas that run, uploaded.
    void build_lists()
    {
        // kernel variant: 1 when any replica has per-site data, 2 when any
        // has exchange tensors or cubic anisotropy
        int variant = 0;
        for (const auto& sl : slots_) {
            if (!sl.used)
                continue;
            if (sl.rec.flags & kVariant2Flags)
                variant = 2;
            else if ((sl.rec.flags & kGeneralFlags) && variant < 1)
                variant = 1;
        }
        if (variant != variant_)
            drop_graph();
        variant_ = variant;
        resident_ = resident_v_[variant_];
        // fused step: every replica of the batch can take it, with one block
        // size and one number of sites per cell
        bool fused = fused_on_;
        int f_nb = -1, f_bt = -1, f_kind = -1, f_plane = 0;
        for (const auto& sl : slots_) {
            if (!sl.used || !fused)
                continue;
            if (!(sl.rec.flags & kFused) || !sl.rec.f_partials)
                fused = false;
            else if ((f_nb >= 0 && f_nb != sl.lat.nb) || (f_bt >= 0 && f_bt != sl.fshape.bt) ||
                     (f_kind >= 0 && f_kind != sl.lat.kind))
                fused = false;
            f_nb = sl.lat.nb;
            f_bt = sl.fshape.bt;
            f_kind = sl.lat.kind;
            f_plane = std::max(f_plane, fused_plane_bytes(sl.fshape, sl.lat.nb, sizeof(R)));
        }
        // two-launch tiles (the Monte Carlo records take them in fused mode too)
        work_.clear();
        for (size_t q = 0; q < slots_.size(); ++q)
                if (slots_[q].used && slots_[q].rec.nsteps > 0)
                    for (int32_t b : tile_order(slots_[q].rec.blocks, order_ ? slots_[q].plane_tiles : 0,
                                                group_ > 0 ? group_
                                                           : balanced_group(slots_[q].plane_tiles, slots_[q].rec.tile)))
                        work_.push_back(WorkItem{(int32_t)q, b});
        fwork_.clear();
        if (fused)
            for (size_t q = 0; q < slots_.size(); ++q)
                if (slots_[q].used && slots_[q].rec.nsteps > 0)
                    fwork_.insert(fwork_.end(), slots_[q].f_items.begin(), slots_[q].f_items.end());
        if (fused != fused_mode_ || f_nb != fused_nb_ || f_bt != fused_bt_ || f_kind != fused_kind_ ||
            f_plane != fused_plane_)
            drop_graph();
        fused_mode_ = fused;
        fused_nb_ = f_nb;
        fused_bt_ = f_bt;
        fused_kind_ = f_kind;
        fused_plane_ = f_plane;
        if (fused) {
            const int nf = (int)fwork_.size();
            if (nf > fwork_cap_ || !d_fwork_) {
                drop_graph();
                (void)hipFree(d_fwork_);
                d_fwork_ = nullptr;
                fwork_cap_ = std::max<int64_t>(std::max(nf, 1), 2 * fwork_cap_);
                hip_check(hipMalloc(&d_fwork_, sizeof(FusedItem) * (size_t)fwork_cap_ + sizeof(int)),
                          "hipMalloc(fused work)");
            }
            int res = 1 << 30;
            for (const auto& sl : slots_)
                if (sl.used)
                    res = std::min(res, fused_resident(sl.lat, sl.fshape));
            const int64_t cap = std::max<int64_t>(8, ((int64_t)(res * grid_scale_) + 7) & ~int64_t(7));
            const int fgrid = nf == 0 ? 0 : (int)std::min<int64_t>(((int64_t)nf + 7) & ~int64_t(7), cap);
            if (fgrid != fgrid_)
                drop_graph();
            fgrid_ = fgrid;
            if (nf > 0)
                hip_check(hipMemcpy(d_fwork_, fwork_.data(), sizeof(FusedItem) * (size_t)nf, hipMemcpyHostToDevice),
                          "upload fused work");
            hip_check(hipMemcpy(reinterpret_cast<char*>(d_fwork_) + sizeof(FusedItem) * (size_t)fwork_cap_, &nf,
                                sizeof(int), hipMemcpyHostToDevice),
                      "upload fused work");
        }
        const int nwork = (int)work_.size();
        if (nwork > work_cap_) {
            drop_graph();
            (void)hipFree(d_work_);
            d_work_ = nullptr;
            work_cap_ = std::max<int64_t>(nwork, 2 * work_cap_);
            hip_check(hipMalloc(&d_work_, sizeof(WorkItem) * (size_t)work_cap_), "hipMalloc(work)");
        }
        // Launch grid: the tiles are swept by at most as many workgroups as
        // fit on the device at once (a multiple of 8 for the XCD mapping).
        // A changing batch always launches the full resident grid so that
        // one captured graph serves every batch.
        const int64_t cap = std::max<int64_t>(8, ((int64_t)(resident_ * grid_scale_) + 7) & ~int64_t(7));
        int grid = (int)std::min<int64_t>(((int64_t)nwork + 7) & ~int64_t(7), cap);
        if (round_grid_)
            grid = resident_;
        if (nwork == 0)
            grid = 0;
        if (grid != grid_)
            drop_graph();
        grid_ = grid;
        if (!work_.empty())
            hip_check(hipMemcpy(d_work_, work_.data(), sizeof(WorkItem) * work_.size(), hipMemcpyHostToDevice),
                      "upload work");
        hip_check(hipMemcpy(d_nwork_, &nwork, sizeof(int), hipMemcpyHostToDevice), "upload nwork");
    }

    // Run one chunk of K launch steps; replica q advances mirror(q).nsteps
    // (<= K) steps.  With use_graph the launch sequence is captured once per
    // (K, grid) and replayed.
    void run_chunk(int K, hipStream_t st, bool use_graph)
    {
        sync_tables(st);
        last_stream_ = st;
        if (grid_ > 0) {
            if (use_graph) {
                if (!graph_exec_ || graph_K_ != K) {
                    drop_graph();
                    hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
                    hipError_t e = enqueue(K, st);
                    hipGraph_t g = nullptr;
                    hipError_t e2 = hipStreamEndCapture(st, &g);
                    hip_check(e, "capture launches");
                    hip_check(e2, "end capture");
                    hipError_t e3 = hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    hip_check(e3, "graph instantiate");
                    graph_K_ = K;
                    ++graph_captures_;
                }
                hip_check(hipGraphLaunch(graph_exec_, st), "graph launch");
            } else {
                hip_check(enqueue(K, st), "kernel launch");
            }
        }
        // host mirror follows the device-side advance
        for (auto& sl : slots_) {
            if (!sl.used || sl.rec.nsteps <= 0)
                continue;
            const int ns = sl.rec.nsteps;
            sl.rec.step += (uint64_t)ns;
            sl.rec.parity = (sl.rec.parity + ns) & 1;
            if (sl.rec.flags & kRecordSeries)
                sl.rec.rec_pos += ns;
        }
    }

    // Monte Carlo: one sweep (every colour class in turn) over replica q's
    // current state, numbered `step` for the random-number counters.
    void mc_sweep(int q, uint64_t step, double cone, double inv_kT, unsigned long long* accepted, hipStream_t st)
    {
        sync_tables();
        last_stream_ = st;
        const Slot& sl = slots_[q];
        if (!sl.d_colour)
            fail(SLLG_E_STATE, "the replica has no colour classes");
        for (size_t c = 0; c + 1 < sl.colour_start.size(); ++c)
            hip_check(launch_mc<R>(d_reps_ + q, sl.d_colour + sl.colour_start[c],
                                   sl.d_colour_pid ? sl.d_colour_pid + sl.colour_start[c] : nullptr,
                                   (int)(sl.colour_start[c + 1] - sl.colour_start[c]), step, cone, inv_kT,
                                   accepted, (sl.rec.flags & kTensor) != 0, st),
                      "Monte Carlo sweep");
    }

    // m and E of the current state of every recording replica that takes
    // part in the work list into record slot `slot`.
    void record_current(int slot, hipStream_t st)
    {
        sync_tables();
        last_stream_ = st;
        if (fused_mode_ && fgrid_ > 0) {
            // the fused step's measuring plane walk over the state in place
            // (k = -1), then the items' sums into the slot
            const int* nf =
                (const int*)(reinterpret_cast<const char*>(d_fwork_) + sizeof(FusedItem) * (size_t)fwork_cap_);
            hip_check(launch_fused<R>(d_reps_, d_fwork_, nf, fgrid_, -1, remap_, true, true, fused_kind_, fused_nb_,
                                      fused_bt_, fused_plane_, st),
                      "measure");
            hip_check(launch_fused_record<R>(d_reps_, (int)slots_.size(), slot, st), "record");
            return;
        }
        if (grid_ <= 0)
            return;
        hip_check(launch_predict<R>(d_reps_, d_work_, d_nwork_, grid_, 1, remap_, true, variant_, st),
                  "measure");
        hip_check(launch_finish<R>(d_reps_, (int)slots_.size(), 1, slot, st), "finish record");
    }

    // Macrocell demagnetising field of replica q from its current state
    // (queued on st).
    void demag_update(int q, hipStream_t st)
    {
        sync_tables();
        last_stream_ = st;
        hip_check(launch_demag<R>(d_reps_ + q, slots_[q].rec.dm_cells, slots_[q].rec.dm_chunks, st),
                  "demagnetising field");
    }

    // The field of the last update, per macrocell (3 per cell).
    void demag_fetch(int q, std::vector<double>& out, hipStream_t st)
    {
        const ReplicaDev<R>& r = slots_[q].rec;
        std::vector<R> tmp(3 * (size_t)r.dm_cells);
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        quiesce();
        hip_check(hipMemcpy(tmp.data(), r.dm_field, tmp.size() * sizeof(R), hipMemcpyDeviceToHost),
                  "download demagnetising field");
        out.assign(tmp.begin(), tmp.end());
    }

    // Replace the held field of replica q (3 per cell, tesla).
    void demag_set(int q, const std::vector<double>& in)
    {
        const ReplicaDev<R>& r = slots_[q].rec;
        if (in.size() != 3 * (size_t)r.dm_cells)
            fail(SLLG_E_ARG, "demagnetising field of the wrong size");
        std::vector<R> tmp(in.begin(), in.end());
        quiesce();
        hip_check(hipMemcpy(r.dm_field, tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice),
                  "upload demagnetising field");
    }

    // Largest torque |S_i x H_i| over the sites of every used replica's
    // current state (deterministic field, no thermal term): out[q] per slot.
    void max_torque(std::vector<double>& out, hipStream_t st)
    {
        sync_tables();
        last_stream_ = st;
        std::vector<WorkItem> all;
        for (size_t q = 0; q < slots_.size(); ++q)
            if (slots_[q].used)
                for (int b = 0; b < slots_[q].rec.blocks; ++b)
                    all.push_back(WorkItem{(int32_t)q, b});
        out.assign(slots_.size(), 0.0);
        if (all.empty())
            return;
        if (all.size() != torque_work_.size() ||
            std::memcmp(all.data(), torque_work_.data(), all.size() * sizeof(WorkItem)) != 0) {
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            (void)hipFree(d_torque_work_);
            d_torque_work_ = nullptr;
            hip_check(hipMalloc(&d_torque_work_, sizeof(WorkItem) * all.size() + sizeof(int)), "hipMalloc(torque)");
            const int n = (int)all.size();
            hip_check(hipMemcpy(d_torque_work_, all.data(), sizeof(WorkItem) * all.size(), hipMemcpyHostToDevice),
                      "upload torque work");
            hip_check(hipMemcpy((char*)d_torque_work_ + sizeof(WorkItem) * all.size(), &n, sizeof(int),
                                hipMemcpyHostToDevice),
                      "upload torque work");
            torque_work_ = std::move(all);
        }
        if (!d_torque_)
            hip_check(hipMalloc(&d_torque_, sizeof(double) * slots_.size()), "hipMalloc(torque)");
        const int n = (int)torque_work_.size();
        const int* d_n = (const int*)((const char*)d_torque_work_ + sizeof(WorkItem) * torque_work_.size());
        hip_check(launch_torque<R>(d_reps_, d_torque_work_, d_n, std::min(n, resident_), (int)slots_.size(), variant_,
                                   d_torque_, st),
                  "torque");
        hip_check(hipMemcpyAsync(out.data(), d_torque_, sizeof(double) * slots_.size(), hipMemcpyDeviceToHost, st),
                  "download torque");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    }

    // m and E of every recording replica's current state into records[rec_pos].
    void measure_now(hipStream_t st)
    {
        sync_tables();
        quiesce();
        // all used replicas, whatever their nsteps, take part
        std::vector<WorkItem> all;
        for (size_t q = 0; q < slots_.size(); ++q)
            if (slots_[q].used && (slots_[q].rec.flags & kRecord))
                for (int b = 0; b < slots_[q].rec.blocks; ++b)
                    all.push_back(WorkItem{(int32_t)q, b});
        if (all.empty())
            return;
        WorkItem* d_all = nullptr;
        int* d_n = nullptr;
        hip_check(hipMalloc(&d_all, sizeof(WorkItem) * all.size()), "hipMalloc(measure)");
        hip_check(hipMalloc(&d_n, sizeof(int)), "hipMalloc(measure)");
        const int n = (int)all.size();
        hipError_t e = hipMemcpy(d_all, all.data(), sizeof(WorkItem) * all.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(d_n, &n, sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_predict<R>(d_reps_, d_all, d_n, n, 1, 0, true, variant_, st);
        if (e == hipSuccess)
            e = launch_finish<R>(d_reps_, (int)slots_.size(), 1, 0, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        (void)hipFree(d_all);
        (void)hipFree(d_n);
        hip_check(e, "measure");
    }

    void set_remap(int v)
    {
        if (v != remap_)
            drop_graph();
        remap_ = v;
    }
    int remap() const { return remap_; }
    // HIP graphs captured so far (a chunk that captured one also timed the capture)
    int64_t graph_captures() const { return graph_captures_; }
    // Neighbour spins through the LDS tile window (default) or all straight
    // from global memory; results are the same bit for bit.
    void set_window(bool on)
    {
        if (on != window_) {
            window_ = on;
            mark_dirty();
        }
    }
    // Tile listing: 0 in site order, 1 plane-swept column groups of
    // `group` tiles (lattices with a detected plane stride); group 0 sizes
    // the groups from the L2 capacity.
    void set_tile_order(int order, int group)
    {
        if (order != order_ || group != group_) {
            order_ = order;
            group_ = group;
            mark_dirty();
        }
    }
    void set_round_grid(bool v) { round_grid_ = v; }
    // Workgroups per launch as a multiple of the resident grid (the tiles are
    // swept by that many workgroups; more than resident lets the hardware
    // schedule them, fewer keeps each on its XCD range longer).
    void set_grid_scale(double f)
    {
        if (f != grid_scale_) {
            grid_scale_ = f;
            mark_dirty();
        }
    }
    double grid_scale() const { return grid_scale_; }
    // Copy the current spins of replica q to / from a device scratch buffer.
    void save_spins(int q, void* dst, hipStream_t st)
    {
        const ReplicaDev<R>& r = slots_[q].rec;
        hip_check(hipMemcpyAsync(dst, r.S[r.parity], 3 * (size_t)r.n * sizeof(R), hipMemcpyDeviceToDevice, st),
                  "save spins");
    }
    void load_spins(int q, const void* src, hipStream_t st)
    {
        const ReplicaDev<R>& r = slots_[q].rec;
        hip_check(hipMemcpyAsync(r.S[r.parity], src, 3 * (size_t)r.n * sizeof(R), hipMemcpyDeviceToDevice, st),
                  "restore spins");
    }
    int grid() const { return grid_; }
    int n_replica_slots() const { return (int)slots_.size(); }

private:
    hipError_t enqueue(int K, hipStream_t st)
    {
        const int nrep = (int)slots_.size();
        hipError_t e = hipSuccess;
        if (fused_mode_) {
            // one launch per step, a measuring launch for the chunk's last
            // record, then the records and the advance
            const int* nf = (const int*)(reinterpret_cast<const char*>(d_fwork_) + sizeof(FusedItem) * (size_t)fwork_cap_);
            // the first step of a chunk leaves no record sums, so it never
            // needs the record code
            for (int k = 0; k < K && e == hipSuccess; ++k)
                e = launch_fused<R>(d_reps_, d_fwork_, nf, fgrid_, k, remap_, false, fused_rec_ && k >= 1, fused_kind_,
                                    fused_nb_, fused_bt_, fused_plane_, st);
            if (e == hipSuccess)
                e = launch_fused<R>(d_reps_, d_fwork_, nf, fgrid_, 0, remap_, true, true, fused_kind_, fused_nb_,
                                    fused_bt_, fused_plane_, st);
            if (e == hipSuccess)   // records, averaging sums and the advance
                e = launch_fused_finish<R>(d_reps_, nrep, st);
            return e;
        }
        for (int k = 0; k < K && e == hipSuccess; ++k) {
            e = launch_predict<R>(d_reps_, d_work_, d_nwork_, grid_, k, remap_, false, variant_, st);
            if (e == hipSuccess)
                e = launch_correct<R>(d_reps_, d_work_, d_nwork_, grid_, k, remap_, variant_, st);
        }
        if (e == hipSuccess)
            e = launch_predict<R>(d_reps_, d_work_, d_nwork_, grid_, 0, remap_, true, variant_, st);
        if (e == hipSuccess)
            e = launch_finish<R>(d_reps_, nrep, 0, 0, st);
        if (e == hipSuccess)
            e = launch_accumulate<R>(d_reps_, nrep, st);
        if (e == hipSuccess)
            e = launch_advance<R>(d_reps_, nrep, st);
        return e;
    }

    void drop_graph()
    {
        if (graph_exec_) {
            (void)hipGraphExecDestroy(graph_exec_);
            graph_exec_ = nullptr;
        }
        graph_K_ = -1;
    }

    int device_;
    Allocator* alloc_;
    std::vector<Slot> slots_;
    std::vector<ReplicaDev<R>> host_reps_;
    ReplicaDev<R>* pinned_reps_ = nullptr;   // pinned staging of host_reps_
    std::vector<char> active_;               // replicas in the current work lists (used, nsteps > 0)
    bool lists_dirty_ = true;
    int64_t graph_captures_ = 0;
    std::vector<WorkItem> work_;
    ReplicaDev<R>* d_reps_ = nullptr;
    WorkItem* d_work_ = nullptr;
    int* d_nwork_ = nullptr;
    int64_t work_cap_ = 0;
    int grid_ = 0;
    int resident_ = 0;
    int resident_v_[3] = {0, 0, 0};   // resident workgroups of each kernel variant
    std::vector<WorkItem> torque_work_;   // every tile of every used replica (max_torque)
    WorkItem* d_torque_work_ = nullptr;   // the same list, then its length (int)
    double* d_torque_ = nullptr;          // [slots] largest torque per replica
    int variant_ = 0;                 // kernel variant the batch needs (launch_predict)
    double grid_scale_ = 1.0;
    int remap_ = SLLG_DEFAULT_REMAP;
    // Columns per group sized from the L2 (group_sites_ sites), the plane's
    // columns split evenly.
    int balanced_group(int pt, int tile) const
    {
        const int cap = (int)std::max<int64_t>(1, group_sites_ / std::max(tile, 1));
        if (pt <= cap)
            return std::max(pt, 1);
        const int groups = (pt + cap - 1) / cap;
        return (pt + groups - 1) / groups;
    }

    // fused step
    bool fused_on_ = true;            // option: use it when the whole batch can
    bool fused_mode_ = false;         // the current work list runs it
    int fused_nb_ = -1, fused_bt_ = -1, fused_kind_ = -1, fused_plane_ = 0;
    bool fused_rec_ = true;   // some replica takes records: step launches run the kernel with the record code
    int fgrid_ = 0;
    std::map<int, int> fused_occ_;    // register-limited resident workgroups per (kind, nb, bt)
    size_t lds_limit_ = 0;
    std::vector<FusedItem> fwork_;
    FusedItem* d_fwork_ = nullptr;    // items, then their count (int) at fwork_cap_
    int64_t fwork_cap_ = 0;

    bool window_ = true;
    int order_ = 1;
    int group_ = 0;
    int64_t group_sites_ = 1 << 14;
    bool round_grid_ = false;
    bool dirty_ = true;
    hipGraphExec_t graph_exec_ = nullptr;
    int graph_K_ = -1;
    hipStream_t last_stream_ = nullptr;
};

}  // namespace sllg
