// HIP kernels of libsllg for gfx950 (MI355X): one Heun step of the
// stochastic LLG equation as a predictor launch and a corrector launch over
// every replica of a batch, with in-kernel Philox noise and FP64 block
// reductions of magnetisation and energy.
//
// Paper (Evans et al., arXiv:1310.6143) passages implemented here:
//  - "The classical spin Hamiltonian": exchange, uniaxial anisotropy and
//    Zeeman terms; the effective field H = -(1/mu_s) dH/dS ("Spin Dynamics").
//  - "Langevin Dynamics": thermal field Gamma sqrt(2 lambda kB T/(gamma mu_s dt)).
//  - "Time Integration of the LLG Equation": the Heun predictor on every
//    spin (renormalised), then the corrector on every spin from the original
//    spin with the mean slope (renormalised), the thermal field held fixed
//    within the step.  The launch boundary between the two kernels is the
//    global "all predictors before any corrector" barrier.
//
// Data layout (see layout.hpp): spins are xyz-interleaved (3 reals per
// site).  Neighbours are stencil patterns (a uint8 pattern id per site, the
// patterns' (offset, J) lists in LDS) or SELL-64 (a slice of 64 consecutive
// rows is stored column-major, so lane l of a wavefront reads entry k of its
// row at nb[slice_off + 64 k + l]; each entry packs type << 28 | column).
// A workgroup integrates a tile of consecutive sites; it first copies the
// tile's spins and a halo on either side into LDS with 16-byte loads, reads
// the near links of every row (listed first) from there and only the far
// ones from global memory.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "layout.hpp"
#include "device_common.hpp"

// Build-time tuning of the step kernels: gather-loop unroll depth.
#ifndef SLLG_GATHER_UNROLL
#define SLLG_GATHER_UNROLL 4
#endif
// Near (LDS) gathers per unrolled step.
#ifndef SLLG_NEAR_UNROLL
#define SLLG_NEAR_UNROLL 4
#endif
#ifndef SLLG_WAVES_F32
#define SLLG_WAVES_F32 6
#endif
#ifndef SLLG_WAVES_F64
#define SLLG_WAVES_F64 4
#endif
#ifndef SLLG_WAVES_F32_PS
#define SLLG_WAVES_F32_PS 5
#endif
#ifndef SLLG_WAVES_F64_PS
#define SLLG_WAVES_F64_PS 3
#endif
#ifndef SLLG_WAVES_F32_GEN
#define SLLG_WAVES_F32_GEN 4
#endif
#ifndef SLLG_WAVES_F64_GEN
#define SLLG_WAVES_F64_GEN 2
#endif
// Waves per SIMD the step kernels are compiled for: as many as their LDS
// allows (register use is capped to match).  Kernel variant V: 0 uniform
// material, 1 per-site materials and easy axes, 2 general (also exchange
// tensors and cubic anisotropy).
#define SLLG_STEP_ATTRS                                                                        \
    __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(                       \
        sizeof(R) == 4 ? (V == 0 ? SLLG_WAVES_F32 : V == 1 ? SLLG_WAVES_F32_PS : SLLG_WAVES_F32_GEN)   \
                       : (V == 0 ? SLLG_WAVES_F64 : V == 1 ? SLLG_WAVES_F64_PS : SLLG_WAVES_F64_GEN))))
#define SLLG_PRAGMA(x) _Pragma(#x)
#define SLLG_UNROLL(n) SLLG_PRAGMA(unroll n)

namespace sllg {
namespace {

using namespace dev;

// Spins are read through buffer descriptors: a 32-bit byte offset per
// lane instead of a 64-bit address, and hardware bounds (an offset past the
// buffer reads 0).  The offsets of a stencil pattern are byte offsets.
typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v3i __attribute__((ext_vector_type(3)));
typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t spin_rsrc(const void* base, int n)
{
    // 0x00020000: dword 3 of a raw (untyped) buffer descriptor on gfx9
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, n, 0x00020000);
}

__device__ __forceinline__ V3<float> bload3(__amdgpu_buffer_rsrc_t rs, int off, float)
{
    const v3i v = __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0);
    return V3<float>{__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z)};
}

__device__ __forceinline__ V3<double> bload3(__amdgpu_buffer_rsrc_t rs, int off, double)
{
    const v4i a = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    const v2i b = __builtin_amdgcn_raw_buffer_load_b64(rs, off + 16, 0, 0);
    auto d = [](int lo, int hi) {
        return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
    };
    return V3<double>{d(a.x, a.y), d(a.z, a.w), d(b.x, b.y)};
}

// Neighbour tables a workgroup stages in LDS: the J table and, for the
// stencil layout, every pattern entry as (byte offset of the neighbour's spin
// from the site's own, J of the link).
template <typename R>
struct PatEntry;
template <>
struct PatEntry<float> {
    int32_t off;
    float J;
};
template <>
struct PatEntry<double> {
    int32_t off;
    int32_t pad;
    double J;
};

template <typename R>
struct Shared {
    R jt[kMaxTypes + 1];   // jt[kMaxTypes] = 0: the wide form's padding entries
    uint16_t pat_start[kMaxPatterns + 1];
    uint16_t pat_far[kMaxPatterns];
    PatEntry<R> pat[kMaxPatternEntries];
    // exchange tensors (kTensor): jm[type], jm[kMaxTypes] = 0 for padding
    // entries, and the type of every pattern entry
    R jm[kMaxTypes + 1][9];
    uint8_t ptype[kMaxPatternEntries];
};

// The tile being integrated: spins of sites [i0 - halo, i0 + tile + halo)
// and the tile's pattern ids.
template <typename R>
struct TileLds {
    static constexpr int kWindow = tile_sites<R>() + 2 * kHaloCap;
    alignas(16) R win[3 * kWindow];
    alignas(16) uint8_t pid[tile_sites<R>()];
};

// Caller synchronises before (tables may still be read) and after.
template <typename R, bool TX>
__device__ __forceinline__ void stage_tables(const ReplicaDev<R>& r, Shared<R>& sh)
{
    if (threadIdx.x <= kMaxTypes)
        sh.jt[threadIdx.x] = threadIdx.x < kMaxTypes ? r.jt[threadIdx.x] : (R)0;
    const bool tensor = TX && (r.flags & kTensor);
    if (tensor && threadIdx.x < (kMaxTypes + 1) * 9) {
        const int t = threadIdx.x / 9, q = threadIdx.x % 9;
        sh.jm[t][q] = t < kMaxTypes ? r.jm[t][q] : (R)0;
    }
    if (r.flags & kStencil) {
        const int np = r.n_patterns;
        for (int q = threadIdx.x; q <= np; q += kBlockThreads)
            sh.pat_start[q] = gload(r.pat_start, q);
        for (int q = threadIdx.x; q < np; q += kBlockThreads)
            sh.pat_far[q] = gload(r.pat_far, q);
        const int ne = gload(r.pat_start, np);
        for (int q = threadIdx.x; q < ne; q += kBlockThreads) {
            const int32_t raw = gload(r.pat_tab, q);
            sh.pat[q].off = (raw >> 4) * (int)(3 * sizeof(R));
            sh.pat[q].J = (raw >> 4) != 0 ? r.jt[raw & 15] : (R)0;   // offset 0: padding
            if (tensor)
                sh.ptype[q] = (raw >> 4) != 0 ? (uint8_t)(raw & 15) : (uint8_t)kMaxTypes;
        }
    }
}

// 16-byte chunks [skip, skip + lim) of dst come from memory at base, the
// others are zero.
__device__ __forceinline__ void stage_chunks(const void* base, int skip, int lim, int nc, v4i* dst)
{
    const __amdgpu_buffer_rsrc_t rs = spin_rsrc(base, lim * 16);
    for (int q = threadIdx.x; q < nc; q += kBlockThreads) {
        const int c = q - skip;
        v4i v = {0, 0, 0, 0};
        if (c >= 0 && c < lim)
            v = __builtin_amdgcn_raw_buffer_load_b128(rs, c * 16, 0, 0);
        dst[q] = v;
    }
}

// Spins of window sites [wb, wb + wn) (wb and wn multiples of 4, so every
// chunk boundary is a site-group boundary); sites outside the replica read
// as zero and are never used.
template <typename R>
__device__ __forceinline__ void stage_window(const R* __restrict__ S, int n, int wb, int wn, R* win)
{
    constexpr int kSiteBytes = 3 * (int)sizeof(R);
    const int first = wb < 0 ? 0 : wb;
    const int skip = (first - wb) * kSiteBytes / 16;
    const int nc = wn * kSiteBytes / 16;
    const int64_t avail = (int64_t)spin_buffer_bytes(n, sizeof(R)) - (int64_t)first * kSiteBytes;
    const int lim = (int)min<int64_t>(avail > 0 ? avail / 16 : 0, (int64_t)(nc - skip));
    stage_chunks(S + 3 * (int64_t)first, skip, lim, nc, (v4i*)win);
}

__device__ __forceinline__ void stage_ids(const uint8_t* __restrict__ pid, int n, int i0, int T, uint8_t* dst)
{
    const int nc = T / 16;
    const int64_t avail = (((int64_t)n + 15) & ~int64_t(15)) - i0;
    const int lim = (int)min<int64_t>(avail / 16, (int64_t)nc);
    stage_chunks(pid + i0, 0, lim, nc, (v4i*)dst);
}

template <typename R>
__device__ __forceinline__ V3<R> wload3(const R* win, int byte_off)
{
    const R* p = (const R*)((const char*)win + byte_off);
    return V3<R>{p[0], p[1], p[2]};
}


// x * 3 * sizeof(R) for 0 <= x < 2^24 (a 24-bit multiply is full rate, a
// 32-bit one quarter rate).
template <typename R>
__device__ __forceinline__ int site_bytes(int x)
{
    return (int)__umul24((unsigned)x, 3u * (unsigned)sizeof(R));
}

// Links per batch of the long-row SELL gathers.
constexpr int kSellBatch = 8;

// h += M S_j for a 3x3 row-major coupling matrix M.
template <typename R>
__device__ __forceinline__ void add_link(V3<R>& h, const R* M, const V3<R>& sj)
{
    h.x += M[0] * sj.x + M[1] * sj.y + M[2] * sj.z;
    h.y += M[3] * sj.x + M[4] * sj.y + M[5] * sj.z;
    h.z += M[6] * sj.x + M[7] * sj.y + M[8] * sj.z;
}

// h += (coupling of a link) S_j: the scalar J, or with exchange tensors
// (TX and kTensor) the matrix of the link's type.
template <typename R, bool TX>
__device__ __forceinline__ void add_coupled(V3<R>& h, bool tensor, const Shared<R>& sh, int type, R J,
                                            const V3<R>& sj)
{
    if (TX && tensor) {
        add_link(h, sh.jm[type], sj);
    } else {
        h.x += J * sj.x;
        h.y += J * sj.y;
        h.z += J * sj.z;
    }
}

// sum_k J_k S[j_k] over the neighbours of site i (tile position l, window
// base site wb): the near part from the window, the far part from global
// memory, each in the row's order, then near + far.  `overlap` runs while
// the far gathers are in flight.  TX: exchange tensors allowed (general
// kernel variant).
template <typename R, bool TX, typename F>
__device__ __forceinline__ V3<R> exchange_sum(const ReplicaDev<R>& r, const R* __restrict__ S,
                                              const Shared<R>& sh, const TileLds<R>& tl, int i, int l,
                                              int wb, int wbyte, F&& overlap)
{
    V3<R> hn{0, 0, 0}, hf{0, 0, 0};
    const bool tensor = TX && (r.flags & kTensor);
    if (r.flags & kWide) {
        // Wide stencil: entry k of the site's pattern p at w_tab[k * patterns
        // + p], read through the L2 (the lanes of a wavefront, neighbouring
        // sites, mostly share a few patterns with adjacent numbers); near
        // links from the window, far ones from global memory, each part in
        // the row's order, a batch of kWideBatch entries and then their
        // spins in flight together.  Both parts are padded to whole batches
        // (type kMaxTypes, J = 0), so no batch is cut short.  Byte offsets
        // fit in 31 bits in this form.
        const __amdgpu_buffer_rsrc_t rs = spin_rsrc(S, r.n * (int)(3 * sizeof(R)));
        const int ib = (i - l) * (int)(3 * sizeof(R)) + site_bytes<R>(l);
        const int p = (int)gload(r.w_pid, i);
        const int nn = (int)gload(r.w_near, p), len = r.w_len;
        const int32_t* __restrict__ tab = r.w_tab + p;
        const int64_t np = r.n_patterns;
        overlap();
        for (int k = 0; k < nn; k += kWideBatch) {
            int32_t raw[kWideBatch];
#pragma unroll
            for (int u = 0; u < kWideBatch; ++u)
                raw[u] = gload(tab, (int64_t)(k + u) * np);
#pragma unroll
            for (int u = 0; u < kWideBatch; ++u) {
                const int off = (raw[u] >> 5) * (int)(3 * sizeof(R)), t = raw[u] & 31;
                const V3<R> sj = (r.flags & kDirect) ? bload3(rs, ib + off, R(0)) : wload3(tl.win, wbyte + off);
                add_coupled<R, TX>(hn, tensor, sh, t, sh.jt[t], sj);
            }
        }
        for (int k = nn; k < len; k += kWideBatch) {
            int32_t raw[kWideBatch];
#pragma unroll
            for (int u = 0; u < kWideBatch; ++u)
                raw[u] = gload(tab, (int64_t)(k + u) * np);
            V3<R> sj[kWideBatch];
#pragma unroll
            for (int u = 0; u < kWideBatch; ++u)
                sj[u] = bload3(rs, ib + (raw[u] >> 5) * (int)(3 * sizeof(R)), R(0));
#pragma unroll
            for (int u = 0; u < kWideBatch; ++u)
                add_coupled<R, TX>(hf, tensor, sh, raw[u] & 31, sh.jt[raw[u] & 31], sj[u]);
        }
    } else if (r.flags & kStencil) {
        // byte offsets fit in 31 bits in the stencil form
        const __amdgpu_buffer_rsrc_t rs = spin_rsrc(S, r.n * (int)(3 * sizeof(R)));
        const int ib = (i - l) * (int)(3 * sizeof(R)) + site_bytes<R>(l);
        const int p = tl.pid[l];
        const int b = sh.pat_start[p], f = sh.pat_far[p], e = sh.pat_start[p + 1];
        // The first kFarRegs far gathers are issued before anything else,
        // so their latency overlaps the rest.  Every pattern has at least
        // kFarRegs far entries (padding: offset 0, J = 0, which adds J * S_i
        // = 0 and keeps the sum's value) unless none has any.
        const bool far = !(r.flags & kNoFar);
        const PatEntry<R>* fp = sh.pat + f;
        V3<R> fr[kFarRegs];
        if (far) {
#pragma unroll
            for (int q = 0; q < kFarRegs; ++q)
                fr[q] = bload3(rs, ib + fp[q].off, R(0));
        }
        overlap();
        if (r.flags & kDirect) {   // same terms, same order, from global memory
            SLLG_UNROLL(SLLG_GATHER_UNROLL)
            for (int k = b; k < f; ++k) {
                const PatEntry<R> pe = sh.pat[k];
                const V3<R> sj = bload3(rs, ib + pe.off, R(0));
                add_coupled<R, TX>(hn, tensor, sh, TX ? sh.ptype[k] : 0, pe.J, sj);
            }
        } else {
            SLLG_UNROLL(SLLG_NEAR_UNROLL)
            for (int k = b; k < f; ++k) {
                const PatEntry<R> pe = sh.pat[k];
                const V3<R> sj = wload3(tl.win, wbyte + pe.off);
                add_coupled<R, TX>(hn, tensor, sh, TX ? sh.ptype[k] : 0, pe.J, sj);
            }
        }
        if (far) {
#pragma unroll
            for (int q = 0; q < kFarRegs; ++q)
                add_coupled<R, TX>(hf, tensor, sh, TX ? sh.ptype[f + q] : 0, fp[q].J, fr[q]);
        }
        SLLG_UNROLL(SLLG_GATHER_UNROLL)
        for (int k = f + kFarRegs; k < e; ++k) {
            const PatEntry<R> pe = sh.pat[k];
            const V3<R> sj = bload3(rs, ib + pe.off, R(0));
            add_coupled<R, TX>(hf, tensor, sh, TX ? sh.ptype[k] : 0, pe.J, sj);
        }
    } else {
        overlap();
        const int64_t base = gload(r.slice_off, i >> 6) + (i & 63);
        const uint32_t dw = gload(r.deg, i);
        const int d = (int)(dw & 0xFFFFu), nn = (int)(dw >> 16);
        // Rows of a few dozen links: one link at a time.  Long rows
        // (kLongRows, long-range exchange; general variant only):
        // kSellBatch entries, then their spins, all in flight together,
        // added in row order (an entry past the row's end repeats the last
        // one with a zero coupling).
        const bool batched = TX && (r.flags & kLongRows);
        if (!batched) {
#pragma unroll 2
            for (int k = nn; k < d; ++k) {
                const uint32_t e = gload(r.nb, base + (int64_t)k * kSlice);
                const V3<R> sj = load3(S, (int64_t)(e & kColMask));
                add_coupled<R, TX>(hf, tensor, sh, (int)(e >> kColBits), sh.jt[e >> kColBits], sj);
            }
        } else {
            for (int k = nn; k < d; k += kSellBatch) {
                uint32_t ent[kSellBatch];
#pragma unroll
                for (int u = 0; u < kSellBatch; ++u)
                    ent[u] = gload(r.nb, base + (int64_t)(k + u < d ? k + u : d - 1) * kSlice);
                V3<R> sj[kSellBatch];
#pragma unroll
                for (int u = 0; u < kSellBatch; ++u)
                    sj[u] = load3(S, (int64_t)(ent[u] & kColMask));
#pragma unroll
                for (int u = 0; u < kSellBatch; ++u) {
                    const int t = k + u < d ? (int)(ent[u] >> kColBits) : kMaxTypes;
                    add_coupled<R, TX>(hf, tensor, sh, t, t < kMaxTypes ? sh.jt[t] : (R)0, sj[u]);
                }
            }
        }
        if (!batched) {
            SLLG_UNROLL(SLLG_NEAR_UNROLL)
            for (int k = 0; k < nn; ++k) {
                const uint32_t e = gload(r.nb, base + (int64_t)k * kSlice);
                const V3<R> sj = (r.flags & kDirect) ? load3(S, (int64_t)(e & kColMask))
                                                     : wload3(tl.win, site_bytes<R>((int)(e & kColMask) - wb));
                add_coupled<R, TX>(hn, tensor, sh, (int)(e >> kColBits), sh.jt[e >> kColBits], sj);
            }
        } else {
            for (int k = 0; k < nn; k += kSellBatch) {
                uint32_t ent[kSellBatch];
#pragma unroll
                for (int u = 0; u < kSellBatch; ++u)
                    ent[u] = gload(r.nb, base + (int64_t)(k + u < nn ? k + u : nn - 1) * kSlice);
#pragma unroll
                for (int u = 0; u < kSellBatch; ++u) {
                    const int c = (int)(ent[u] & kColMask);
                    const V3<R> sj = (r.flags & kDirect) ? load3(S, (int64_t)c) : wload3(tl.win, site_bytes<R>(c - wb));
                    const int t = k + u < nn ? (int)(ent[u] >> kColBits) : kMaxTypes;
                    add_coupled<R, TX>(hn, tensor, sh, t, t < kMaxTypes ? sh.jt[t] : (R)0, sj);
                }
            }
        }
    }
    return V3<R>{hn.x + hf.x, hn.y + hf.y, hn.z + hf.z};
}


// ---------------------------------------------------------------------------
// Reductions of m and E, in FP64.  Every sum has a fixed order: sites of a
// tile (the sites of each lane in turn, then by row of 16 lanes, wavefront),
// tiles of a group (kGroupTiles, by tile), groups (by group).  Which workgroup computes a sum never changes
// its order, so a step's record is the same bit for bit whatever the launch
// shape, the chunking or the rest of the batch.
// ---------------------------------------------------------------------------
constexpr int kWaves = kBlockThreads / 64;

// Block-wide sum of four values in a fixed order; result valid in thread 0.
// Ends with a barrier so `red` can be reused at once.
__device__ __forceinline__ void block_sum4(const double v[4], double out[4], double (*red)[kWaves])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double w = wave_sum(v[c]);
        if (lane == 0)
            red[c][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w)
                s += red[c][w];
            out[c] = s;
        }
    }
    __syncthreads();
}

// Group g of a replica's tile partials -> group partial g.
template <typename R>
__device__ void group_reduce(const ReplicaDev<R>& r, int g, double (*red)[kWaves])
{
    const int lo = g * kGroupTiles;
    const int cnt = min(kGroupTiles, r.blocks - lo);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if ((int)threadIdx.x < cnt) {
        const double* p = r.partials + 4 * (int64_t)(lo + (int)threadIdx.x);
#pragma unroll
        for (int c = 0; c < 4; ++c)
            v[c] = p[c];
    }
    double out[4];
    block_sum4(v, out, red);
    if (threadIdx.x == 0) {
        double* q = r.group_partials + 4 * (int64_t)g;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            q[c] = out[c];
    }
}

// All group partials -> record `slot` (m = sum mu S / sum mu, E).
template <typename R>
__device__ void final_reduce(const ReplicaDev<R>& r, int slot, double (*red)[kWaves])
{
    const int n_groups = (r.blocks + kGroupTiles - 1) / kGroupTiles;
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < n_groups; q0 += kBlockThreads) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        const int q = q0 + (int)threadIdx.x;
        if (q < n_groups) {
            const double* p = r.group_partials + 4 * (int64_t)q;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                v[c] = p[c];
        }
        double out[4];
        block_sum4(v, out, red);
        if (threadIdx.x == 0)
            for (int c = 0; c < 4; ++c)
                tot[c] += out[c];
    }
    if (threadIdx.x == 0) {
        double* out = r.records + 4 * (r.rec_pos + slot);
        const double f = r.mu_ref * r.inv_mu_total;
        out[0] = tot[0] * f;
        out[1] = tot[1] * f;
        out[2] = tot[2] * f;
        out[3] = -r.mu_ref * tot[3];
    }
}

template <typename R>
__device__ __forceinline__ MaterialDev<R> site_material(const ReplicaDev<R>& r, int i)
{
    const int q = (r.flags & kPerSiteMaterial) ? gload(r.matid, i) : 0;
    const SLLG_GLOBAL MaterialDev<R>& g = ((const SLLG_GLOBAL MaterialDev<R>*)r.mat)[q];
    MaterialDev<R> m;
    m.mu_rel = g.mu_rel;
    m.mu_frac = g.mu_frac;
    m.ani = g.ani;
    m.ku_mu = g.ku_mu;
    m.sigma = g.sigma;
    m.axis[0] = g.axis[0];
    m.axis[1] = g.axis[1];
    m.axis[2] = g.axis[2];
    m.cub = g.cub;
    m.kc_mu = g.kc_mu;
    m.mu_s = g.mu_s;
    return m;
}

template <typename R>
__device__ __forceinline__ V3<R> site_axis(const ReplicaDev<R>& r, const MaterialDev<R>& m, int i)
{
    if (r.flags & kPerSiteAxis)
        return load3(r.axis, i);
    return V3<R>{m.axis[0], m.axis[1], m.axis[2]};
}

// Sx^4 + Sy^4 + Sz^4.
template <typename R>
__device__ __forceinline__ R quartic(const V3<R>& s)
{
    const R x2 = s.x * s.x, y2 = s.y * s.y, z2 = s.z * s.z;
    return x2 * x2 + y2 * y2 + z2 * z2;
}

// Adds the cubic anisotropy field -(2 k_c/mu_s)(Sx^3, Sy^3, Sz^3).
template <typename R>
__device__ __forceinline__ void add_cubic(const MaterialDev<R>& m, const V3<R>& s, V3<R>& h)
{
    h.x += m.cub * s.x * s.x * s.x;
    h.y += m.cub * s.y * s.y * s.y;
    h.z += m.cub * s.z * s.z * s.z;
}

// Adds the demagnetising field of the site's macrocell (last update).
template <typename R>
__device__ __forceinline__ void add_demag(const ReplicaDev<R>& r, int i, V3<R>& h)
{
    const V3<R> f = load3((const R*)r.dm_field, (int64_t)gload(r.dm_cell, i));
    h.x += f.x;
    h.y += f.y;
    h.z += f.z;
}

// Adds the thermal field sigma * g (normals g drawn for this site and step).
template <typename R>
__device__ __forceinline__ void add_thermal(const MaterialDev<R>& m, const R g[3], V3<R>& h)
{
    if (m.sigma != (R)0) {
        h.x += m.sigma * g[0];
        h.y += m.sigma * g[1];
        h.z += m.sigma * g[2];
    }
}

// ---------------------------------------------------------------------------
// Predictor.  For step k of the chunk: reads S (current state), writes the
// predicted spin S' = |S + dS dt| (the corrector rebuilds S + dS dt / 2 from
// S and S', and draws the step's thermal normals again from their counter).
// With MEASURE it only evaluates m and E: of the state after the chunk's
// steps (k == 0) or of the current state (k == 1).
//
// Records: the state the predictor reads at step k >= 1 is the state after
// step k - 1, and its exchange field is at hand, so the predictor leaves
// per-tile partials of m and E for record k - 1; the corrector of the same
// step sums them by groups, and the tile-0 workgroup of the next predictor
// (or of the measuring pass at the end of the chunk) adds the groups into
// the record.  The chunk's last record is completed by k_finish.
// ---------------------------------------------------------------------------
// The sites of one tile (PS: per-site materials or axes; otherwise the
// material is read once into scalar registers).
template <typename R, bool MEASURE, int V>
__device__ __forceinline__ void predict_sites(const ReplicaDev<R>& r, const R* __restrict__ S,
                                              const Shared<R>& sh, const TileLds<R>& tl, int i0, int wb,
                                              int k, bool partials, double v[4])
{
    constexpr bool PS = V != 0, TX = V == 2;
    const int T = r.tile;
    const MaterialDev<R> m0 = PS ? MaterialDev<R>{} : uniform_material(r);
    for (int l = (int)threadIdx.x; l < T; l += kBlockThreads) {
        const int i = i0 + l;
        if (i >= r.n)
            break;
        const MaterialDev<R> m = PS ? site_material(r, i) : m0;   // loaded before the gathers are issued
        const int wbyte = site_bytes<R>(l + r.halo);
        const V3<R> s = (r.flags & kDirect) ? load3(S, i) : wload3(tl.win, wbyte);
        R g[3] = {0, 0, 0};
        const V3<R> sum = exchange_sum<R, TX>(r, S, sh, tl, i, l, wb, wbyte, [&] {
            if (!MEASURE && m.sigma != (R)0)
                thermal_normals(r.seed, r.step + (uint64_t)k, (uint32_t)i, g);
        });
        const V3<R> hex{m.mu_rel * sum.x, m.mu_rel * sum.y, m.mu_rel * sum.z};
        const V3<R> e = PS ? site_axis(r, m, i) : V3<R>{m.axis[0], m.axis[1], m.axis[2]};
        const R se = dot(s, e);
        const V3<R> Happ{r.H[0], r.H[1], r.H[2]};
        const bool cubic = TX && (r.flags & kCubic);
        if (partials) {
            // in units of mu_ref: mu_s/mu_ref S and mu_s/mu_ref (-E_i/mu_s)
            v[0] += (double)(m.mu_frac * s.x);
            v[1] += (double)(m.mu_frac * s.y);
            v[2] += (double)(m.mu_frac * s.z);
            R u = (R)0.5 * dot(s, hex) + m.ku_mu * se * se + dot(s, Happ);
            if (cubic)
                u -= (R)0.5 * m.kc_mu * quartic(s);
            v[3] += (double)(m.mu_frac * u);
        }
        if (!MEASURE) {
            V3<R> h{hex.x + m.ani * se * e.x + Happ.x, hex.y + m.ani * se * e.y + Happ.y,
                    hex.z + m.ani * se * e.z + Happ.z};
            if (cubic)
                add_cubic(m, s, h);
            if (TX && (r.flags & kDemag))
                add_demag(r, i, h);
            add_thermal(m, g, h);
            const V3<R> ds = llg_step(s, h, r.gdt, r.alpha);
            const V3<R> sp = normalised(V3<R>{s.x + ds.x, s.y + ds.y, s.z + ds.z});
            store3(r.Sp, i, sp);
        }
    }
}

template <typename R, bool MEASURE, int V>
__global__ SLLG_STEP_ATTRS void k_predict(const ReplicaDev<R>* __restrict__ reps,
                                          const WorkItem* __restrict__ work,
                                          const int* __restrict__ n_work, int k, int remap)
{
    __shared__ Shared<R> sh;
    __shared__ TileLds<R> tl;
    __shared__ double red[4][kWaves];
    const int W = *n_work;
    int staged = -1;
    for (TileIter it(W, remap); it.more(); it.next()) {
        const WorkItem w = work[it.t];
        const ReplicaDev<R>& r = reps[w.replica];
        const int nsteps = r.nsteps;
        if (MEASURE ? (!(r.flags & kRecord) || (k == 0 && nsteps <= 0)) : (k >= nsteps))
            continue;   // uniform over the block
        const bool recording = (r.flags & kRecord) != 0;
        const bool partials = recording && (MEASURE || k >= 1);
        const int par = (r.parity + (MEASURE ? (k == 0 ? nsteps : 0) : k)) & 1;
        const R* __restrict__ S = r.S[par];
        const int T = r.tile;
        const int i0 = w.block * T, wb = i0 - r.halo;
        __syncthreads();   // every lane is done with the previous tile's LDS
        if (w.replica != staged) {
            stage_tables<R, V == 2>(r, sh);
            staged = w.replica;
        }
        if (!(r.flags & kDirect))
            stage_window(S, r.n, wb, T + 2 * r.halo, tl.win);
        if (r.flags & kStencil)
            stage_ids(r.pat_id, r.n, i0, T, tl.pid);
        __syncthreads();
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (V != 0 && (r.flags & kGeneralFlags))
            predict_sites<R, MEASURE, V>(r, S, sh, tl, i0, wb, k, partials, v);
        else
            predict_sites<R, MEASURE, 0>(r, S, sh, tl, i0, wb, k, partials, v);
        if (partials) {
            double out[4];
            block_sum4(v, out, red);
            if (threadIdx.x == 0) {
                double* p = r.partials + 4 * (int64_t)w.block;
                p[0] = out[0];
                p[1] = out[1];
                p[2] = out[2];
                p[3] = out[3];
            }
        }
        // group partials left by the previous corrector -> their record
        if (recording && w.block == 0) {
            if (!MEASURE && k >= 2)
                final_reduce(r, k - 2, red);
            else if (MEASURE && k == 0 && nsteps >= 2)
                final_reduce(r, nsteps - 2, red);
        }
    }
}

// ---------------------------------------------------------------------------
// Corrector.  Field at S' with the same thermal numbers (same counter),
// slope dS', and S_new = |S + (dS + dS') dt / 2| written to the other
// ping-pong buffer.  The predictor's increment is not stored: dS is
// perpendicular to S and |S| = 1, so the site's own predictor
// S' = (S + dS dt)/|S + dS dt| has S.S' = 1/|S + dS dt|, and
// S + dS dt / 2 = (S + S'/(S.S'))/2 comes from S and S' (whatever the
// rounding of the predictor's normalisation, which cancels in S'/(S.S')).
// Workgroups whose tile opens a group of kGroupTiles also sum that group of
// the predictor's partials.
// ---------------------------------------------------------------------------

template <typename R, int V>
__device__ __forceinline__ void correct_sites(const ReplicaDev<R>& r, const R* __restrict__ Sc,
                                              const R* __restrict__ Sp, R* __restrict__ Sn,
                                              const Shared<R>& sh, const TileLds<R>& tl, int i0, int wb,
                                              int k)
{
    constexpr bool PS = V != 0, TX = V == 2;
    const int T = r.tile;
    const MaterialDev<R> m0 = PS ? MaterialDev<R>{} : uniform_material(r);
    for (int l = (int)threadIdx.x; l < T; l += kBlockThreads) {
        const int i = i0 + l;
        if (i >= r.n)
            break;
        const MaterialDev<R> m = PS ? site_material(r, i) : m0;   // loaded before the gathers are issued
        const int wbyte = site_bytes<R>(l + r.halo);
        const V3<R> sp = (r.flags & kDirect) ? load3(Sp, i) : wload3(tl.win, wbyte);
        const V3<R> s0 = load3_once(Sc, i);
        R g[3] = {0, 0, 0};
        const V3<R> sum = exchange_sum<R, TX>(r, Sp, sh, tl, i, l, wb, wbyte, [&] {
            if (m.sigma != (R)0)
                thermal_normals(r.seed, r.step + (uint64_t)k, (uint32_t)i, g);
        });
        const V3<R> e = PS ? site_axis(r, m, i) : V3<R>{m.axis[0], m.axis[1], m.axis[2]};
        const R se = dot(sp, e);
        V3<R> h{m.mu_rel * sum.x + m.ani * se * e.x + r.H[0],
                m.mu_rel * sum.y + m.ani * se * e.y + r.H[1],
                m.mu_rel * sum.z + m.ani * se * e.z + r.H[2]};
        if (TX && (r.flags & kCubic))
            add_cubic(m, sp, h);
        if (TX && (r.flags & kDemag))
            add_demag(r, i, h);
        add_thermal(m, g, h);
        const V3<R> ds = llg_step(sp, h, r.gdt, r.alpha);
        const R q = (R)0.5 * recip(dot(s0, sp));
        const V3<R> b{(R)0.5 * s0.x + q * sp.x, (R)0.5 * s0.y + q * sp.y, (R)0.5 * s0.z + q * sp.z};
        const V3<R> sn = normalised(V3<R>{b.x + (R)0.5 * ds.x, b.y + (R)0.5 * ds.y, b.z + (R)0.5 * ds.z});
        store3(Sn, i, sn);
        if (!spin_ok(sn))
            flag_fault(r.fault);
    }
}

template <typename R, int V>
__global__ SLLG_STEP_ATTRS void k_correct(const ReplicaDev<R>* __restrict__ reps,
                                          const WorkItem* __restrict__ work,
                                          const int* __restrict__ n_work, int k, int remap)
{
    __shared__ Shared<R> sh;
    __shared__ TileLds<R> tl;
    __shared__ double red[4][kWaves];
    const int W = *n_work;
    int staged = -1;
    for (TileIter it(W, remap); it.more(); it.next()) {
        const WorkItem w = work[it.t];
        const ReplicaDev<R>& r = reps[w.replica];
        if (k >= r.nsteps)
            continue;
        const R* __restrict__ Sp = r.Sp;
        const int T = r.tile;
        const int i0 = w.block * T, wb = i0 - r.halo;
        __syncthreads();   // every lane is done with the previous tile's LDS
        if (w.replica != staged) {
            stage_tables<R, V == 2>(r, sh);
            staged = w.replica;
        }
        if (!(r.flags & kDirect))
            stage_window(Sp, r.n, wb, T + 2 * r.halo, tl.win);
        if (r.flags & kStencil)
            stage_ids(r.pat_id, r.n, i0, T, tl.pid);
        __syncthreads();
        const R* __restrict__ Sc = r.S[(r.parity + k) & 1];
        R* __restrict__ Sn = r.S[(r.parity + k + 1) & 1];
        if (V != 0 && (r.flags & kGeneralFlags))
            correct_sites<R, V>(r, Sc, Sp, Sn, sh, tl, i0, wb, k);
        else
            correct_sites<R, 0>(r, Sc, Sp, Sn, sh, tl, i0, wb, k);
        if ((r.flags & kRecord) && k >= 1 && (w.block % kGroupTiles) == 0)
            group_reduce(r, w.block / kGroupTiles, red);
    }
}

// The last record of a chunk (mode 0) or the current state's (mode 1, into
// record slot `slot`): all groups, then the total, by one workgroup per
// replica, in the same order as the per-step path.
template <typename R>
__global__ __launch_bounds__(kBlockThreads) void k_finish(const ReplicaDev<R>* __restrict__ reps, int mode,
                                                          int slot)
{
    __shared__ double red[4][kWaves];
    const ReplicaDev<R>& r = reps[blockIdx.x];
    if (!(r.flags & kRecord) || (mode == 0 && r.nsteps <= 0))
        return;
    const int n_groups = (r.blocks + kGroupTiles - 1) / kGroupTiles;
    for (int g = 0; g < n_groups; ++g)
        group_reduce(r, g, red);
    __threadfence_block();
    __syncthreads();
    final_reduce(r, mode == 0 ? r.nsteps - 1 : slot, red);
}

// ---------------------------------------------------------------------------
// Torque ("Angular variation of the coercivity": the LLG equation is solved
// until the torque |S x H_eff| on the system is small).  k_torque: per tile,
// the largest |S_i x H_i| of the current state with the deterministic field
// (exchange, anisotropy, applied field; no thermal term) into
// partials[4 * tile]; k_torque_max: the largest over each replica's tiles.
// The maximum does not depend on the order, so the result is exact and
// reproducible.
// ---------------------------------------------------------------------------
template <typename R, int V>
__device__ __forceinline__ double torque_sites(const ReplicaDev<R>& r, const R* __restrict__ S,
                                               const Shared<R>& sh, const TileLds<R>& tl, int i0, int wb)
{
    constexpr bool PS = V != 0, TX = V == 2;
    const int T = r.tile;
    const MaterialDev<R> m0 = PS ? MaterialDev<R>{} : uniform_material(r);
    double worst = 0.0;
    for (int l = (int)threadIdx.x; l < T; l += kBlockThreads) {
        const int i = i0 + l;
        if (i >= r.n)
            break;
        const MaterialDev<R> m = PS ? site_material(r, i) : m0;
        const int wbyte = site_bytes<R>(l + r.halo);
        const V3<R> s = (r.flags & kDirect) ? load3(S, i) : wload3(tl.win, wbyte);
        const V3<R> sum = exchange_sum<R, TX>(r, S, sh, tl, i, l, wb, wbyte, [] {});
        const V3<R> e = PS ? site_axis(r, m, i) : V3<R>{m.axis[0], m.axis[1], m.axis[2]};
        const R se = dot(s, e);
        V3<R> h{m.mu_rel * sum.x + m.ani * se * e.x + r.H[0], m.mu_rel * sum.y + m.ani * se * e.y + r.H[1],
                m.mu_rel * sum.z + m.ani * se * e.z + r.H[2]};
        if (TX && (r.flags & kCubic))
            add_cubic(m, s, h);
        if (TX && (r.flags & kDemag))
            add_demag(r, i, h);
        const V3<R> t{s.y * h.z - s.z * h.y, s.z * h.x - s.x * h.z, s.x * h.y - s.y * h.x};
        worst = fmax(worst, (double)sqrt(dot(t, t)));
    }
    return worst;
}

// Largest value over the block; result valid in thread 0.  Ends with a barrier.
__device__ __forceinline__ double block_max(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kWaves; ++w)
            m = fmax(m, red[w]);
    __syncthreads();
    return m;
}

template <typename R, int V>
__global__ SLLG_STEP_ATTRS void k_torque(const ReplicaDev<R>* __restrict__ reps, const WorkItem* __restrict__ work,
                                         const int* __restrict__ n_work, int remap)
{
    __shared__ Shared<R> sh;
    __shared__ TileLds<R> tl;
    __shared__ double red[kWaves];
    const int W = *n_work;
    int staged = -1;
    for (TileIter it(W, remap); it.more(); it.next()) {
        const WorkItem w = work[it.t];
        const ReplicaDev<R>& r = reps[w.replica];
        const R* __restrict__ S = r.S[r.parity];
        const int T = r.tile;
        const int i0 = w.block * T, wb = i0 - r.halo;
        __syncthreads();   // every lane is done with the previous tile's LDS
        if (w.replica != staged) {
            stage_tables<R, V == 2>(r, sh);
            staged = w.replica;
        }
        if (!(r.flags & kDirect))
            stage_window(S, r.n, wb, T + 2 * r.halo, tl.win);
        if (r.flags & kStencil)
            stage_ids(r.pat_id, r.n, i0, T, tl.pid);
        __syncthreads();
        const double worst = (V != 0 && (r.flags & kGeneralFlags)) ? torque_sites<R, V>(r, S, sh, tl, i0, wb)
                                                                   : torque_sites<R, 0>(r, S, sh, tl, i0, wb);
        const double m = block_max(worst, red);
        if (threadIdx.x == 0)
            r.partials[4 * (int64_t)w.block] = m;
    }
}

// One workgroup per replica: the largest tile value -> out[replica].
template <typename R>
__global__ __launch_bounds__(kBlockThreads) void k_torque_max(const ReplicaDev<R>* __restrict__ reps,
                                                              double* __restrict__ out)
{
    __shared__ double red[kWaves];
    const ReplicaDev<R>& r = reps[blockIdx.x];
    double v = 0.0;
    for (int b = (int)threadIdx.x; b < r.blocks; b += kBlockThreads)
        v = fmax(v, r.partials[4 * (int64_t)b]);
    const double m = block_max(v, red);
    if (threadIdx.x == 0)
        out[blockIdx.x] = m;
}

// ---------------------------------------------------------------------------
// Macrocell demagnetising field ("Demagnetising fields").  k_demag_moments:
// m_p = sum over the cell's sites of mu_s,i S_i, one thread per cell, sites
// in a fixed order.  k_demag_field: for every cell p,
//   H_p = mu0/(4 pi) sum_{q != p} [3 (m_q . r) r - m_q] / |x_q - x_p|^3
//         - (mu0/3) m_p / V_p,
// one thread per cell p, the cells q staged through LDS a workgroup's width
// at a time (all-pairs: the work is n_cells^2 pair terms, the data n_cells
// moments and positions).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_demag_moments(const ReplicaDev<R>* __restrict__ rep)
{
    const ReplicaDev<R>& r = *rep;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= r.dm_cells)
        return;
    const R* __restrict__ S = r.S[r.parity];
    const int b = gload(r.dm_start, p), e = gload(r.dm_start, p + 1);
    double m[3] = {0.0, 0.0, 0.0};
    for (int k = b; k < e; ++k) {
        const int i = gload(r.dm_atoms, k);
        const double mu = site_material(r, i).mu_s;
        const V3<R> s = load3(S, i);
        m[0] += mu * (double)s.x;
        m[1] += mu * (double)s.y;
        m[2] += mu * (double)s.z;
    }
    store3(r.dm_m, p, V3<R>{(R)m[0], (R)m[1], (R)m[2]});
}

constexpr int kDemagBlock = 256;

// 1/sqrt: the hardware reciprocal square root in FP32, exact division in FP64.
__device__ __forceinline__ float inv_sqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

// Partial dipole sums: block (bx, c) takes cells p of block bx and the
// sources q of chunk c, staged through LDS; dm_part[c] receives the sums.
template <typename R>
__global__ __launch_bounds__(kDemagBlock) void k_demag_pairs(const ReplicaDev<R>* __restrict__ rep)
{
    __shared__ R tile[6][kDemagBlock];
    const ReplicaDev<R>& r = *rep;
    const int nc = r.dm_cells;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < nc;
    const int per = (nc + r.dm_chunks - 1) / r.dm_chunks;
    const int qb = (int)blockIdx.y * per, qe = min(nc, qb + per);
    const V3<R> xp = live ? load3(r.dm_pos, p) : V3<R>{0, 0, 0};
    R hx = 0, hy = 0, hz = 0;
    for (int q0 = qb; q0 < qe; q0 += kDemagBlock) {
        const int q = q0 + (int)threadIdx.x;
        __syncthreads();
        if (q < qe) {
            const V3<R> x = load3(r.dm_pos, q), m = load3((const R*)r.dm_m, q);
            tile[0][threadIdx.x] = x.x;
            tile[1][threadIdx.x] = x.y;
            tile[2][threadIdx.x] = x.z;
            tile[3][threadIdx.x] = m.x;
            tile[4][threadIdx.x] = m.y;
            tile[5][threadIdx.x] = m.z;
        }
        __syncthreads();
        const int cnt = min(kDemagBlock, qe - q0);
        for (int k = 0; k < cnt; ++k) {
            const R dx = tile[0][k] - xp.x, dy = tile[1][k] - xp.y, dz = tile[2][k] - xp.z;
            const R mx = tile[3][k], my = tile[4][k], mz = tile[5][k];
            const bool self = q0 + k == p;
            const R r2 = self ? (R)1 : dx * dx + dy * dy + dz * dz;
            const R inv = inv_sqrt(r2);
            const R inv2 = inv * inv;
            const R inv3 = self ? (R)0 : inv2 * inv;
            const R md = (R)3 * (mx * dx + my * dy + mz * dz) * inv2;   // 3 (m . r) / |d| with r = d / |d|
            hx += (md * dx - mx) * inv3;
            hy += (md * dy - my) * inv3;
            hz += (md * dz - mz) * inv3;
        }
    }
    if (live) {
        R* part = r.dm_part + 3 * (int64_t)nc * blockIdx.y;
        store3(part, p, V3<R>{hx, hy, hz});
    }
}

// Chunk sums in chunk order, scaled by mu0 / (4 pi), plus the self term.
template <typename R>
__global__ __launch_bounds__(256) void k_demag_field(const ReplicaDev<R>* __restrict__ rep)
{
    const ReplicaDev<R>& r = *rep;
    const int nc = r.dm_cells;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nc)
        return;
    R hx = 0, hy = 0, hz = 0;
    for (int c = 0; c < r.dm_chunks; ++c) {
        const V3<R> h = load3((const R*)r.dm_part + 3 * (int64_t)nc * c, p);
        hx += h.x;
        hy += h.y;
        hz += h.z;
    }
    const V3<R> mp = load3((const R*)r.dm_m, p);
    const R self = gload(r.dm_self, p);
    const R k = (R)1e-7;   // mu0 / (4 pi), T m / A
    store3(r.dm_field, p, V3<R>{k * hx - self * mp.x, k * hy - self * mp.y, k * hz - self * mp.z});
}

// End of a chunk: advance the step counter and the ping-pong parity.
template <typename R>
__global__ void k_advance(ReplicaDev<R>* __restrict__ reps, int n_rep)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_rep)
        advance_replica(reps[j]);
}

template <typename R>
__global__ void k_noise(uint64_t seed, uint64_t step, int n, double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        R g[3];
        thermal_normals(seed, step, (uint32_t)i, g);
        out[3 * i] = (double)g[0];
        out[3 * i + 1] = (double)g[1];
        out[3 * i + 2] = (double)g[2];
    }
}

// ---------------------------------------------------------------------------
// Monte Carlo ("Monte Carlo Methods"): one Metropolis trial with a
// Hinzke-Nowak move on every site of one colour class of a greedy colouring
// of the neighbour graph.  Sites of a class share no link, so their trials
// are independent and can run at once, in place.  Move type (flip,
// Gaussian in a cone of width sigma_g, uniform on the sphere) and the
// acceptance uniform come from Philox counter (site, step lo, step hi, 3),
// the Gaussian numbers from counter (site, step lo, step hi, 2).
// ---------------------------------------------------------------------------

// sum_k J_k S[j_k] / mu_ref over the neighbours of site i, the spins
// straight from global memory.  Pattern tables come from LDS (the wide
// form's from global memory); neighbours are taken kMcBatch at a time, every load of a batch issued before the first is
// used (entries past the end repeat the last one with J = 0), and added in
// table order.
constexpr int kMcBatch = 8;
// FP32 Monte Carlo grid: at most this many times the resident workgroups
// (measured on the bcc block: 1, 2 and 4 give 0.21, 0.194 and 0.22 ms per
// four-class sweep; one workgroup per chunk 0.242 ms)
constexpr int kMcResidentFactor = 2;

template <typename R, bool TX>
__device__ __forceinline__ V3<R> exchange_sum_global(const ReplicaDev<R>& r, const Shared<R>& sh,
                                                     const R* __restrict__ S, int i, int p)
{
    V3<R> h{0, 0, 0};
    const char* sb = (const char*)S;
    const bool tensor = TX && (r.flags & kTensor);
    if (r.flags & kWide) {
        // the pattern's entries in table order (near links, then far ones;
        // padding entries have J = 0)
        const int len = r.w_len;
        const int32_t* __restrict__ tab = r.w_tab + p;
        const int64_t np = r.n_patterns;
        const char* si = sb + (int64_t)i * (3 * sizeof(R));
        for (int k = 0; k < len; k += kWideBatch) {
            int32_t raw[kWideBatch];
#pragma unroll
            for (int u = 0; u < kWideBatch; ++u)
                raw[u] = gload(tab, (int64_t)(k + u) * np);
            V3<R> sj[kWideBatch];
#pragma unroll
            for (int u = 0; u < kWideBatch; ++u)
                sj[u] = load3((const R*)(si + (int64_t)(raw[u] >> 5) * (int64_t)(3 * sizeof(R))), 0);
#pragma unroll
            for (int u = 0; u < kWideBatch; ++u)
                add_coupled<R, TX>(h, tensor, sh, raw[u] & 31, sh.jt[raw[u] & 31], sj[u]);
        }
        return h;
    }
    if (r.flags & kStencil) {
        const int b = sh.pat_start[p], e = sh.pat_start[p + 1];
        const char* si = sb + (int64_t)i * (3 * sizeof(R));
        for (int k = b; k < e; k += kMcBatch) {
            V3<R> sj[kMcBatch];
            R J[kMcBatch];
            int ty[kMcBatch];
#pragma unroll
            for (int u = 0; u < kMcBatch; ++u) {
                const int kk = k + u < e ? k + u : e - 1;
                const PatEntry<R> pe = sh.pat[kk];
                J[u] = k + u < e ? pe.J : (R)0;
                ty[u] = tensor ? (k + u < e ? (int)sh.ptype[kk] : kMaxTypes) : 0;
                sj[u] = load3((const R*)(si + pe.off), 0);
            }
#pragma unroll
            for (int u = 0; u < kMcBatch; ++u)
                add_coupled<R, TX>(h, tensor, sh, ty[u], J[u], sj[u]);
        }
        return h;
    }
    const int64_t base = gload(r.slice_off, i >> 6) + (i & 63);
    const int d = (int)(gload(r.deg, i) & 0xFFFFu);
    for (int k = 0; k < d; k += kMcBatch) {
        uint32_t ent[kMcBatch];
#pragma unroll
        for (int u = 0; u < kMcBatch; ++u)
            ent[u] = gload(r.nb, base + (int64_t)(k + u < d ? k + u : d - 1) * kSlice);
        V3<R> sj[kMcBatch];
#pragma unroll
        for (int u = 0; u < kMcBatch; ++u)
            sj[u] = load3(S, (int64_t)(ent[u] & kColMask));
#pragma unroll
        for (int u = 0; u < kMcBatch; ++u) {
            const int t = k + u < d ? (int)(ent[u] >> kColBits) : kMaxTypes;
            add_coupled<R, TX>(h, tensor, sh, t, t < kMaxTypes ? sh.jt[t] : (R)0, sj[u]);
        }
    }
    return h;
}

template <typename R, bool TX>
__global__ __launch_bounds__(kBlockThreads) void k_mc(const ReplicaDev<R>* __restrict__ rep,
                                                      const int32_t* __restrict__ sites,
                                                      const uint16_t* __restrict__ pids, int count, uint64_t step,
                                                      R cone, double inv_kT, unsigned long long* __restrict__ accepted)
{
    __shared__ Shared<R> sh;
    __shared__ unsigned int acc_block;
    const ReplicaDev<R>& r = *rep;
    if (threadIdx.x == 0)
        acc_block = 0;
    stage_tables<R, TX>(r, sh);
    __syncthreads();
    // Workgroups are handed to the 8 XCDs round-robin, and each XCD has its
    // own L2.  Sites of neighbouring chunks of the class list share
    // neighbours (cells one row or plane apart), so XCD x takes a
    // contiguous range of the class's chunks, shared out among its
    // workgroups (those with b mod 8 = x; the grid is a multiple of 8).  In
    // FP32 the grid is capped near the resident workgroups, so a workgroup
    // takes several chunks and stages the tables above once for them.
    const int NC = (count + (int)blockDim.x - 1) / (int)blockDim.x;
    const int q = NC >> 3, rem = NC & 7, x = (int)blockIdx.x & 7;
    const int start = x * q + (x < rem ? x : rem), len = q + (x < rem ? 1 : 0);
    const int per_xcd = (int)gridDim.x >> 3;
    auto trial = [&](int t) {
        // the site and, for the stencil forms, its pattern: two independent
        // loads from lists in the class's order
        const int i = gload(sites, t);
        const int p = pids ? (int)gload(pids, t) : 0;
        R* __restrict__ S = r.S[r.parity];
        const MaterialDev<R> m = site_material(r, i);
        const V3<R> s = load3((const R*)S, i);
        const V3<R> sum = exchange_sum_global<R, TX>(r, sh, (const R*)S, i, p);
        const V3<R> h{m.mu_rel * sum.x + r.H[0], m.mu_rel * sum.y + r.H[1], m.mu_rel * sum.z + r.H[2]};
        uint32_t c0 = (uint32_t)i, c1 = (uint32_t)step, c2 = (uint32_t)(step >> 32), c3 = 3u;
        philox10(c0, c1, c2, c3, (uint32_t)r.seed, (uint32_t)(r.seed >> 32));
        const uint32_t move = (uint32_t)(((uint64_t)c0 * 3u) >> 32);
        const double u = (double)c1 * 2.3283064365386963e-10;
        R g[3];
        thermal_normals(r.seed, step, (uint32_t)i, g, 2u);
        V3<R> tr;
        if (move == 0) {
            tr = V3<R>{-s.x, -s.y, -s.z};
        } else {
            tr = move == 1 ? V3<R>{s.x + cone * g[0], s.y + cone * g[1], s.z + cone * g[2]}
                           : V3<R>{g[0], g[1], g[2]};
            tr = normalised(tr);
        }
        const V3<R> e = site_axis(r, m, i);
        const R se = dot(s, e), te = dot(tr, e);
        // dE = -mu_s [(S' - S).(H_exc + H) + (k_u/mu_s)((S'.e)^2 - (S.e)^2)
        //             - (k_c/(2 mu_s))(S'x^4 + S'y^4 + S'z^4 - Sx^4 - Sy^4 - Sz^4)]
        const V3<R> d{tr.x - s.x, tr.y - s.y, tr.z - s.z};
        R bracket = dot(d, h) + m.ku_mu * (te * te - se * se);
        if (r.flags & kCubic)
            bracket -= (R)0.5 * m.kc_mu * (quartic(tr) - quartic(s));
        // accept when dE <= 0, else with probability exp(-dE/(kB T)); the
        // decision is taken in the kernel's precision
        bool accept = bracket >= (R)0;
        if (!accept && inv_kT > 0.0)
            accept = (R)u < exp(bracket * (R)(m.mu_s * inv_kT));
        if (accept) {
            store3(S, i, tr);
            if (!spin_ok(tr))
                flag_fault(r.fault);
            atomicAdd(&acc_block, 1u);
        }
    };
    if constexpr (sizeof(R) == 4) {
        for (int j = (int)blockIdx.x >> 3; j < len; j += per_xcd) {
            const int t = (start + j) * (int)blockDim.x + (int)threadIdx.x;
            if (t < count)
                trial(t);
        }
    } else {
        // one chunk per workgroup (the grid covers every chunk): the loop
        // would cost the FP64 kernel registers and a wave per SIMD
        const int t = (start + ((int)blockIdx.x >> 3)) * (int)blockDim.x + (int)threadIdx.x;
        if (((int)blockIdx.x >> 3) < len && t < count)
            trial(t);
    }
    __syncthreads();
    if (threadIdx.x == 0 && acc_block)
        atomicAdd(accepted, (unsigned long long)acc_block);
}

// Copy per-step records (m, E) of one replica into caller arrays.
__global__ void k_scatter_records(const double* __restrict__ rec, int count,
                                  double* __restrict__ m_dev, double* __restrict__ E_dev)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) {
        if (m_dev) {
            m_dev[3 * t] = rec[4 * t];
            m_dev[3 * t + 1] = rec[4 * t + 1];
            m_dev[3 * t + 2] = rec[4 * t + 2];
        }
        if (E_dev)
            E_dev[t] = rec[4 * t + 3];
    }
}

// Running block sums for thermal averages, one thread per replica:
// acc[b] += (|m|, m_x, m_y, m_z, E) for every record of this chunk whose
// step falls in averaging block b = (step - avg_first) / avg_block_len.
// Each replica's samples are added one by one in step order, so the sums do
// not depend on the chunking or on the other replicas of the batch.
template <typename R>
__global__ void k_accumulate(const ReplicaDev<R>* __restrict__ reps, int n_rep)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_rep)
        accumulate_records(reps[j]);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
template <typename R>
hipError_t launch_predict(const ReplicaDev<R>* reps, const WorkItem* work, const int* n_work,
                          int grid, int k, int remap, bool measure, int variant, hipStream_t st)
{
    if (grid <= 0)
        return hipSuccess;
    const dim3 g(grid), b(kBlockThreads);
    if (measure) {
        if (variant == 2)
            hipLaunchKernelGGL((k_predict<R, true, 2>), g, b, 0, st, reps, work, n_work, k, remap);
        else if (variant == 1)
            hipLaunchKernelGGL((k_predict<R, true, 1>), g, b, 0, st, reps, work, n_work, k, remap);
        else
            hipLaunchKernelGGL((k_predict<R, true, 0>), g, b, 0, st, reps, work, n_work, k, remap);
    } else {
        if (variant == 2)
            hipLaunchKernelGGL((k_predict<R, false, 2>), g, b, 0, st, reps, work, n_work, k, remap);
        else if (variant == 1)
            hipLaunchKernelGGL((k_predict<R, false, 1>), g, b, 0, st, reps, work, n_work, k, remap);
        else
            hipLaunchKernelGGL((k_predict<R, false, 0>), g, b, 0, st, reps, work, n_work, k, remap);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_correct(const ReplicaDev<R>* reps, const WorkItem* work, const int* n_work,
                          int grid, int k, int remap, int variant, hipStream_t st)
{
    if (grid <= 0)
        return hipSuccess;
    const dim3 g(grid), b(kBlockThreads);
    if (variant == 2)
        hipLaunchKernelGGL((k_correct<R, 2>), g, b, 0, st, reps, work, n_work, k, remap);
    else if (variant == 1)
        hipLaunchKernelGGL((k_correct<R, 1>), g, b, 0, st, reps, work, n_work, k, remap);
    else
        hipLaunchKernelGGL((k_correct<R, 0>), g, b, 0, st, reps, work, n_work, k, remap);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_finish(const ReplicaDev<R>* reps, int n_rep, int mode, int slot, hipStream_t st)
{
    if (n_rep <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_finish<R>), dim3(n_rep), dim3(kBlockThreads), 0, st, reps, mode, slot);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_advance(ReplicaDev<R>* reps, int n_rep, hipStream_t st)
{
    if (n_rep <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_advance<R>), dim3((n_rep + 63) / 64), dim3(64), 0, st, reps, n_rep);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_noise(uint64_t seed, uint64_t step, int n, double* out, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_noise<R>), dim3((n + 255) / 256), dim3(256), 0, st, seed, step, n, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_mc(const ReplicaDev<R>* rep, const int32_t* sites, const uint16_t* pids, int count, uint64_t step,
                     double cone, double inv_kT, unsigned long long* accepted, bool tensor, hipStream_t st)
{
    if (count <= 0)
        return hipSuccess;
    // one workgroup per chunk of kBlockThreads sites, rounded to a multiple
    // of 8 (the XCD share-out in k_mc); FP32: at most kMcResidentFactor
    // times the resident workgroups of the kernel, each then taking several
    // chunks and staging its tables once (FP64 keeps one chunk per
    // workgroup: the chunk loop costs its kernel a wave per SIMD)
    static int resident[2][16];   // per kernel variant and device, 0 = not yet queried
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16)
        return hipErrorInvalidDevice;
    int& res = resident[tensor ? 1 : 0][dev];
    if (res == 0) {
        int cus = 0, per_cu = 0;
        const void* f = tensor ? (const void*)k_mc<R, true> : (const void*)k_mc<R, false>;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlockThreads, 0) != hipSuccess)
            return hipErrorInvalidValue;
        res = (cus * (per_cu > 0 ? per_cu : 1)) & ~7;
        if (res < 8)
            res = 8;
    }
    const int chunks = (count + kBlockThreads - 1) / kBlockThreads;
    const int cap = sizeof(R) == 4 ? res * kMcResidentFactor : 0x7FFFFFF8;
    const int grid = ((chunks + 7) & ~7) < cap ? ((chunks + 7) & ~7) : cap;
    const dim3 g(grid), b(kBlockThreads);
    if (tensor)
        hipLaunchKernelGGL((k_mc<R, true>), g, b, 0, st, rep, sites, pids, count, step, (R)cone, inv_kT, accepted);
    else
        hipLaunchKernelGGL((k_mc<R, false>), g, b, 0, st, rep, sites, pids, count, step, (R)cone, inv_kT, accepted);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_torque(const ReplicaDev<R>* reps, const WorkItem* work, const int* n_work, int grid,
                         int n_rep, int variant, double* out, hipStream_t st)
{
    if (grid <= 0 || n_rep <= 0)
        return hipSuccess;
    const dim3 g(grid), b(kBlockThreads);
    if (variant == 2)
        hipLaunchKernelGGL((k_torque<R, 2>), g, b, 0, st, reps, work, n_work, 0);
    else if (variant == 1)
        hipLaunchKernelGGL((k_torque<R, 1>), g, b, 0, st, reps, work, n_work, 0);
    else
        hipLaunchKernelGGL((k_torque<R, 0>), g, b, 0, st, reps, work, n_work, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_torque_max<R>), dim3(n_rep), b, 0, st, reps, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_demag(const ReplicaDev<R>* rep, int cells, int chunks, hipStream_t st)
{
    if (cells <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_demag_moments<R>), dim3((cells + 255) / 256), dim3(256), 0, st, rep);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_demag_pairs<R>), dim3((cells + kDemagBlock - 1) / kDemagBlock, chunks), dim3(kDemagBlock), 0,
                       st, rep);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_demag_field<R>), dim3((cells + 255) / 256), dim3(256), 0, st, rep);
    return hipGetLastError();
}

template <typename R>
int resident_blocks(int device, int variant)
{
    int cus = 0, a = 0, b = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        return 0;
    const void* kp = variant == 2 ? (const void*)k_predict<R, false, 2>
                     : variant == 1 ? (const void*)k_predict<R, false, 1> : (const void*)k_predict<R, false, 0>;
    const void* kc = variant == 2 ? (const void*)k_correct<R, 2>
                     : variant == 1 ? (const void*)k_correct<R, 1> : (const void*)k_correct<R, 0>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, kp, kBlockThreads, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kc, kBlockThreads, 0) != hipSuccess)
        return 0;
    const int per_cu = a < b ? a : b;
    return cus * (per_cu > 0 ? per_cu : 1);
}

hipError_t launch_scatter_records(const double* rec, int count, double* m_dev, double* E_dev,
                                  hipStream_t st)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_scatter_records, dim3((count + 255) / 256), dim3(256), 0, st, rec, count,
                       m_dev, E_dev);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_accumulate(const ReplicaDev<R>* reps, int n_rep, hipStream_t st)
{
    if (n_rep <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_accumulate<R>), dim3((n_rep + 63) / 64), dim3(64), 0, st, reps, n_rep);
    return hipGetLastError();
}

#define SLLG_INSTANTIATE(R)                                                                          \
    template hipError_t launch_predict<R>(const ReplicaDev<R>*, const WorkItem*, const int*, int, int, \
                                          int, bool, int, hipStream_t);                              \
    template hipError_t launch_correct<R>(const ReplicaDev<R>*, const WorkItem*, const int*, int, int, \
                                          int, int, hipStream_t);                                    \
    template hipError_t launch_accumulate<R>(const ReplicaDev<R>*, int, hipStream_t);                \
    template hipError_t launch_finish<R>(const ReplicaDev<R>*, int, int, int, hipStream_t);         \
    template hipError_t launch_advance<R>(ReplicaDev<R>*, int, hipStream_t);                         \
    template hipError_t launch_noise<R>(uint64_t, uint64_t, int, double*, hipStream_t);             \
    template int resident_blocks<R>(int, int);                                                        \
    template hipError_t launch_demag<R>(const ReplicaDev<R>*, int, int, hipStream_t);                \
    template hipError_t launch_torque<R>(const ReplicaDev<R>*, const WorkItem*, const int*, int, int, int, \
                                         double*, hipStream_t);                                      \
    template hipError_t launch_mc<R>(const ReplicaDev<R>*, const int32_t*, const uint16_t*, int, uint64_t, double, double, \
                                     unsigned long long*, bool, hipStream_t);

SLLG_INSTANTIATE(float)
SLLG_INSTANTIATE(double)

}  // namespace sllg
