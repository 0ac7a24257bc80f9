// Fused Heun step of libsllg for gfx950: one launch per step of the
// stochastic LLG equation on lattices declared cell by cell (sites
// i = b + nb (x + nx (y + ny z)), links between cells at most one cell
// apart on every axis).
//
// Paper (Evans et al., arXiv:1310.6143), "Time Integration of the LLG
// Equation": every spin takes the predictor S' = |S + dS dt| before any
// corrector S <- |S + (dS + dS') dt / 2| uses it, the field re-evaluated
// at S' with the same thermal field ("Langevin Dynamics").  The two-launch
// kernels (kernels.hip) keep that order with a launch boundary.  Here a
// workgroup instead owns a tile of TX x TY cell columns and recomputes the
// predictor on the ring of cells around it, so its corrector needs no other
// workgroup's results, and the step reads S once and writes it once.
//
// Plane marching.  The workgroup walks its columns up through a range of
// planes.  At plane q the spins S(q) of the tile, the ring and one more
// ring sit in LDS; thread (px, py) owns one column of the tile-plus-ring
// region and keeps, in registers, running exchange sums of its sites in the
// planes q - 1, q, q + 1: the links of a site in plane q - 1 that reach
// plane q complete its field, so the predictor of plane q - 1 runs, writes
// S'(q - 1) to another LDS plane, and the same running sums over S' give the
// corrector of plane q - 2.  A site's exchange sum is therefore added in a
// fixed order, links into the plane below, then its own plane, then the
// plane above, each in the canonical link order, whatever the tiling.
// Thermal field, S' and S + dS dt / 2 of a site stay in the registers of
// the thread that owns its column from the predictor to the corrector.
//
// Memory.  S(q + 1) streams into a second LDS plane by direct global-to-LDS
// loads while plane q is worked on (no registers held for it).  For the
// lattice kinds compiled in (simple cubic, bcc, bcc with second
// neighbours) a link's LDS offset is a constant: one LDS read and three
// FMAs per link.  Planes beyond an open z surface are zero, so surface
// sites use the bulk link list (the missing links add J * 0).
//
// Records.  The predictor of step k sees the state after step k - 1 with
// its exchange field, so each item leaves FP64 sums of m and E of that
// state for its own sites; the first item of a replica in the launch of
// step k + 1 adds the items' sums (a fixed order) into record k - 1; a
// measuring launch (the same plane walk without predictor and corrector,
// its third LDS plane holding a third S plane so that each plane's copy
// overlaps the work on the previous ones) and k_fused_finish complete the
// last two of a chunk.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace sllg {
namespace {

using namespace dev;

// FP32 LDS slot of one site: x, y, z and a fourth word (the next site's x
// as it arrives from memory; never used).
struct alignas(16) Slot4 {
    float x, y, z, w;
};
// FP64: x and y of a site (its z sits in the second half of the row).
struct alignas(16) XY64 {
    double x, y;
};
// 16 bytes of zeros: a lane's share of a plane beyond an open surface.
struct alignas(16) Zero16 {
    uint32_t w[4];
};

// Plane layout constants of a precision and block size: the FP64 row width
// in slots (RW) and the distance of a site's z from its x, y (ZOFF); the
// chunks a wave copies per plane (CPW).
template <typename R, int BT>
struct PlaneLayout {
    static constexpr int RW = fused_row_slots(sizeof(R), BT);
    static constexpr int ZOFF = RW * 16;
    static constexpr int CPW = fused_chunks_per_wave(sizeof(R));
};

template <typename R>
using FEnt = std::conditional_t<sizeof(R) == 4, FusedEntry, FusedEntryD>;

typedef __attribute__((address_space(3))) void* lds_ptr;

// Sum of four values over the first 256 threads (fixed order: per wave, then
// the four waves in turn); result valid in thread 0.  Every thread of the
// block calls it.
template <int BT>
__device__ __forceinline__ void sum4_256(const double v[4], double out[4], double (*red)[BT / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double s = wave_sum(threadIdx.x < 256 ? v[c] : 0.0);
        if (lane == 0 && wave < 4)
            red[c][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            out[c] = ((red[c][0] + red[c][1]) + red[c][2]) + red[c][3];
    __syncthreads();
}

// Record `slot` of replica r from its items' sums of parity `par`: thread t
// < 256 adds items t, t + 256, ... in order, then the fixed 256-lane sum.
// The same order whichever kernel runs it.
template <typename R, int BT>
__device__ void fused_record(const ReplicaDev<R>& r, int par, int64_t slot, double (*red)[BT / 64])
{
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const double* p = r.f_partials + 4 * (int64_t)par * r.f_items;
    if (threadIdx.x < 256)
        for (int q = (int)threadIdx.x; q < r.f_items; q += 256) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                v[c] += p[4 * (int64_t)q + c];
        }
    double tot[4];
    sum4_256<BT>(v, tot, red);
    if (threadIdx.x == 0) {
        double* out = r.records + 4 * (r.rec_pos + slot);
        const double f = r.mu_ref * r.inv_mu_total;
        out[0] = tot[0] * f;
        out[1] = tot[1] * f;
        out[2] = tot[2] * f;
        // the Zeeman part from the summed spins: S.H_app summed over the
        // sites is H_app.(sum of S)
        const double zee = (double)r.H[0] * tot[0] + (double)r.H[1] * tot[1] + (double)r.H[2] * tot[2];
        out[3] = -r.mu_ref * (tot[3] + zee);
    }
}

__device__ __forceinline__ int wrap_cell(int u, int n)
{
    const int m = u % n;
    return m < 0 ? m + n : m;
}

// m and E terms of one site: S and S.H_ex/2 + (k_u/mu_s)(S.e)^2, with se =
// S.e as the predictor forms it (-E_i/mu_s is that plus S.H_app, which the
// record adds from the summed spins).  A replica takes the fused step only
// with one material, so mu_s is the reference moment and every site weighs
// 1.  Written with explicit fmas so that the step and the measuring launch
// round alike.
template <typename R>
__device__ __forceinline__ void record_terms(const MaterialDev<R>& m, const V3<R>& s, R se, const V3<R>& hex, R t[4])
{
    const R sh = fma(s.z, hex.z, fma(s.y, hex.y, s.x * hex.x));
    t[0] = s.x;
    t[1] = s.y;
    t[2] = s.z;
    t[3] = fma((R)0.5, sh, m.ku_mu * se * se);
}

// The terms of one cell (its basis sites added in R, in basis order) into
// the thread's own FP64 sums, added in plane order: acc[c * AS].  FP32 keeps
// the sums in LDS (AS = the block size; constant offsets let the four
// read-modify-writes overlap), FP64 in registers (AS = 1: its kernel has
// room below the 256 registers of two waves per SIMD).
template <int AS, typename R>
__device__ __forceinline__ void record_add(const R t[4], double* acc)
{
    double a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        a[c] = acc[c * AS];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        acc[c * AS] = a[c] + (double)t[c];
}

// x, y, z of the LDS slot at p.  FP32: the fourth word is never read; the
// slot is read through its 16-byte-aligned type, so the compiler emits one
// 12-byte LDS read (ds_read_b96) for the three words it uses (through a
// 4-byte-aligned 12-byte type it splits the read into two or three
// instructions, which cost the step a fifth of its time).  FP64: a 16-byte
// read of x, y and an 8-byte read of z, ZOFF bytes further (one address,
// two immediate offsets).
template <typename R, int ZOFF>
__device__ __forceinline__ V3<R> slot_xyz(const char* p)
{
    if constexpr (sizeof(R) == 4) {
        const Slot4 v = *reinterpret_cast<const Slot4*>(p);
        return V3<R>{v.x, v.y, v.z};
    } else {
        const XY64 v = *reinterpret_cast<const XY64*>(p);
        return V3<R>{v.x, v.y, *reinterpret_cast<const double*>(p + ZOFF)};
    }
}

template <typename R, int ZOFF>
__device__ __forceinline__ void slot_store(char* p, const V3<R>& v)
{
    if constexpr (sizeof(R) == 4) {
        *reinterpret_cast<Slot4*>(p) = Slot4{v.x, v.y, v.z, 0.0f};
    } else {
        *reinterpret_cast<XY64*>(p) = XY64{v.x, v.y};
        *reinterpret_cast<double*>(p + ZOFF) = v.z;
    }
}

// Per-thread geometry of an item.  An LDS plane holds the region's sites
// basis-major, row after row (FP32: 16 bytes per site, rows of the region's
// width; FP64: rows of RW sites, x, y then z), so the lanes of a wave read
// consecutive slots and a link's slot is a constant distance away.
template <int NB>
struct ItemGeo {
    int rb[NB][3];      // byte offset of slot (bp, row py + 1 + dy, column px) for dy = -1, 0, 1
    uint32_t col;       // site index of the thread's cell, plane 0, site 0
    uint32_t plane_sites;
    bool live, interior;
    __device__ int own(int b) const { return rb[b][1] + 16; }   // the thread's site b
};

// h += links of basis site b whose dz is DZ, read from the plane at `base`
// (the slots of this thread's cell: rb).  Compiled kinds: constant offsets
// and the two slot couplings kj; generic: pattern p's entries from LDS.
template <typename R, int KIND, int NB, int DZ, int ZOFF>
__device__ __forceinline__ void add_dz(V3<R>& h, const char* __restrict__ base, const ItemGeo<NB>& g, int b,
                                       const R kj[2], const int4* pat, const FEnt<R>* ent, int p)
{
    if constexpr (KIND != kKindGeneric) {
        (void)pat;
        (void)ent;
        (void)p;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
#pragma unroll
                for (int bp = 0; bp < NB; ++bp) {
                    int slot = 0;
                    if (!kind_link(KIND, b, DZ, dy, dx, bp, &slot))
                        continue;
                    const V3<R> v = slot_xyz<R, ZOFF>(base + g.rb[bp][dy + 1] + (dx + 1) * 16);
                    h.x = fma(kj[slot], v.x, h.x);
                    h.y = fma(kj[slot], v.y, h.y);
                    h.z = fma(kj[slot], v.z, h.z);
                }
    } else {
        (void)kj;
        if (p < 0)
            return;
        const int4 hd = pat[p];
        const int first = hd.x + (DZ >= 0 ? hd.y : 0) + (DZ > 0 ? hd.z : 0);
        const int cnt = DZ < 0 ? hd.y : DZ == 0 ? hd.z : hd.w;
        // entry offsets are from the site's own slot
        const char* own = base + g.own(b);
#pragma unroll 4
        for (int q = 0; q < cnt; ++q) {
            const FEnt<R> en = ent[first + q];
            const V3<R> v = slot_xyz<R, ZOFF>(own + en.off);
            h.x = fma((R)en.J, v.x, h.x);
            h.y = fma((R)en.J, v.y, h.y);
            h.z = fma((R)en.J, v.z, h.z);
        }
    }
}

// Whether any link of `kind` (any basis site, any dz) reads slot (dy, dx, bp)
// of a plane.
__host__ __device__ constexpr bool kind_reads(int kind, int dy, int dx, int bp)
{
    for (int b = 0; b < 2; ++b)
        for (int dz = -1; dz <= 1; ++dz) {
            int slot = 0;
            if (b < kind_basis(kind) && kind_link(kind, b, dz, dy, dx, bp, &slot))
                return true;
        }
    return false;
}

// Compiled kinds: every link the thread's sites take from one plane at
// `base`, each distinct slot read once.  hu (sites one plane below, their
// dz = +1 links), h0 (sites of this plane, dz = 0) and hd (sites one plane
// above, dz = -1) receive the sums, each link in the canonical order.
template <typename R, int KIND, int NB, int ZOFF>
__device__ __forceinline__ void plane_links(const char* __restrict__ base, const ItemGeo<NB>& g, const R kj[2],
                                            V3<R> hu[NB], V3<R> h0[NB], V3<R> hd[NB])
{
    V3<R> v[3][3][NB];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
#pragma unroll
            for (int bp = 0; bp < NB; ++bp)
                if (kind_reads(KIND, dy, dx, bp))
                    v[dy + 1][dx + 1][bp] = slot_xyz<R, ZOFF>(base + g.rb[bp][dy + 1] + (dx + 1) * 16);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int dz = 1; dz >= -1; --dz) {
            V3<R>& h = dz > 0 ? hu[b] : dz == 0 ? h0[b] : hd[b];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
#pragma unroll
                    for (int bp = 0; bp < NB; ++bp) {
                        int slot = 0;
                        if (!kind_link(KIND, b, dz, dy, dx, bp, &slot))
                            continue;
                        const V3<R>& u = v[dy + 1][dx + 1][bp];
                        h.x = fma(kj[slot], u.x, h.x);
                        h.y = fma(kj[slot], u.y, h.y);
                        h.z = fma(kj[slot], u.z, h.z);
                    }
        }
}

// Pattern of basis site b in plane z for the generic kind, -1 where the
// plane does not exist.
template <typename R>
__device__ __forceinline__ int plane_pattern(const ReplicaDev<R>& r, int z, int b)
{
    if (r.f_zper)
        z = wrap_cell(z, r.f_nz);
    else if (z < 0 || z >= r.f_nz)
        return -1;
    return r.f_plane ? (int)r.f_plane[z * r.f_nb + b] : b;
}

// Running state of the thread's sites between planes, in two slots chosen
// by the parity of the plane (relative to the item's first), so that a
// value stays in the same registers from the plane step that creates it
// to the one that uses it.
template <typename R, int NB>
struct ColumnState {
    V3<R> hp[2][NB];              // predictor sums of plane p in slot p & 1
    V3<R> hc[2][NB];              // corrector sums of plane p in slot p & 1
    V3<R> c_sp[2][NB], c_base[2][NB], c_th[2][NB];   // S', S + dS dt / 2, thermal + applied field of plane p
};

// Fixed facts of an item for its plane iterations.
template <typename R>
struct ItemRun {
    const R* S;                   // state the step starts from
    R* Sn;                        // state it writes
    const uint32_t* dcol;         // [CPW][BT] byte offset (plane 0) of the 16 bytes each lane copies, or ~0
    __amdgpu_buffer_rsrc_t rsrc;  // the spins S as a buffer (reads past its end return 0)
    int n_chunks;
    int z0, z1;
    bool partials;
    uint64_t step;
};

// One plane step q of an item (P: parity of q relative to the item's
// first plane step): A links from S(q) in `cur` into planes q - 1
// (completing it), q and q + 1; B predictor of plane q - 1 (its spins still
// in `nxt`) into `sp`; barrier; the copy of S(q + 1) into `nxt` is issued
// (direct global-to-LDS loads of 16 bytes per site, or zeros beyond an open
// surface); D links from S'(q - 1) into planes q - 2 (completing it), q - 1
// and q; E corrector of plane q - 2; barrier.  The LDS pointers are distinct planes (restrict), so the
// reads of `cur` and `sp` need not wait for the copy into `nxt`; the
// closing barrier does.
template <typename R, int KIND, int NB, int BT, bool MEASURE, int P, bool REC>
__device__ __forceinline__ void plane_step(const ReplicaDev<R>& r, const ItemGeo<NB>& g, const ItemRun<R>& run,
                                           ColumnState<R, NB>& cs, const char* __restrict__ cur,
                                           char* __restrict__ nxt, char* __restrict__ sp, double* __restrict__ acc,
                                           const int4* pat, const FEnt<R>* ent, int q, int zw_m2, int zw_m1,
                                           int zw_p1, const MaterialDev<R>& m)
{
    constexpr int S0 = P, S1 = P ^ 1;   // slots of planes q (and q - 2, q + 2) and q - 1 (and q + 1)
    constexpr int ZOFF = PlaneLayout<R, BT>::ZOFF, CPW = PlaneLayout<R, BT>::CPW;
    const int nz = r.f_nz;
    const bool zper = r.f_zper != 0;
    const int z0 = run.z0, z1 = run.z1;
    const R kj[2] = {r.f_kj[0], r.f_kj[1]};
    const V3<R> e{m.axis[0], m.axis[1], m.axis[2]};
    const V3<R> Happ{r.H[0], r.H[1], r.H[2]};
    const int zp = q - 1;
    const bool zp_exists = zper || (zp >= 0 && zp < nz);
    const bool zp_need = zp >= z0 - 1 && zp <= z1 && zp_exists;
    const bool zp_own = zp >= z0 && zp < z1;
    // Issue the copy of S(q + 1) into the LDS plane dst: direct
    // global-to-LDS loads of 16 bytes per lane, or zeros beyond an open
    // surface; nothing past the item's last needed plane.  The next barrier
    // completes it.
    auto copy_next = [&](char* __restrict__ dst) {
        if (q + 1 > z1 + 1)
            return;
        const bool exists = zper || (q + 1 >= 0 && q + 1 < nz);
        // the wave number as a scalar: the chunk addresses below are then
        // computed on the scalar unit when needed, not held in registers
        const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int c = wave + j * (BT / 64);
            if (c >= run.n_chunks)
                break;   // uniform over the wave
            char* d = dst + c * 64 * 16;
            const uint32_t dc = run.dcol[j * BT + (int)threadIdx.x];
            if (dc != 0xFFFFFFFFu) {
                if (exists) {
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        run.rsrc, (lds_ptr)d, 16, (int)dc,
                        (int)(g.plane_sites * 3u * (uint32_t)sizeof(R) * (uint32_t)zw_p1), 0, 0);
                } else {
                    reinterpret_cast<Zero16*>(d)[lane] = Zero16{{0u, 0u, 0u, 0u}};
                }
            }
        }
    };
    // The measuring launch holds three S planes (it has no S'): S(q + 1)
    // streams into the free one while S(q) and S(q - 1) are worked on.
    if constexpr (MEASURE)
        copy_next(sp);
    // A: links from S(q) into planes q - 1 (completing it), q and q + 1
    V3<R> up[NB];   // plane q + 1's first sums, moved into the slot of q - 1 after B
#pragma unroll
    for (int b = 0; b < NB; ++b)
        up[b] = V3<R>{0, 0, 0};
    if (g.live) {
        if constexpr (KIND != kKindGeneric) {
            plane_links<R, KIND, NB, ZOFF>(cur, g, kj, cs.hp[S1], cs.hp[S0], up);
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                add_dz<R, KIND, NB, 1, ZOFF>(cs.hp[S1][b], cur, g, b, kj, pat, ent, plane_pattern(r, q - 1, b));
                add_dz<R, KIND, NB, 0, ZOFF>(cs.hp[S0][b], cur, g, b, kj, pat, ent, plane_pattern(r, q, b));
                add_dz<R, KIND, NB, -1, ZOFF>(up[b], cur, g, b, kj, pat, ent, plane_pattern(r, q + 1, b));
            }
        }
    }
    // B: m and E terms of plane q - 1 (its exchange sums are complete; one
    // material: the exchange field is the sum itself) from the spins its
    // predictor reads, then the predictor
    const bool rec = REC && run.partials && g.interior && zp_need && zp_own;
    R tc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (g.live && zp_need) {
            const V3<R> s = slot_xyz<R, ZOFF>(nxt + g.own(b));
            const V3<R>& hex = cs.hp[S1][b];
            const R se = fma(s.z, e.z, fma(s.y, e.y, s.x * e.x));
            if (rec) {
                R t[4];
                record_terms(m, s, se, hex, t);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    tc[c] = b == 0 ? t[c] : tc[c] + t[c];
            }
            if (!MEASURE) {
                R gn[3] = {0, 0, 0};
                if (m.sigma != (R)0)
                    thermal_normals(r.seed, run.step, g.col + (uint32_t)b + g.plane_sites * (uint32_t)zw_m1, gn);
                // thermal plus applied field, held for the corrector
                const V3<R> tha{fma(m.sigma, gn[0], Happ.x), fma(m.sigma, gn[1], Happ.y),
                                fma(m.sigma, gn[2], Happ.z)};
                const R as = m.ani * se;
                const V3<R> h{fma(as, e.x, hex.x) + tha.x, fma(as, e.y, hex.y) + tha.y, fma(as, e.z, hex.z) + tha.z};
                const V3<R> ds = llg_step(s, h, r.gdt, r.alpha);
                const V3<R> spn = normalised(V3<R>{s.x + ds.x, s.y + ds.y, s.z + ds.z});
                cs.c_th[S1][b] = tha;
                cs.c_sp[S1][b] = spn;
                cs.c_base[S1][b] = V3<R>{s.x + (R)0.5 * ds.x, s.y + (R)0.5 * ds.y, s.z + (R)0.5 * ds.z};
                slot_store<R, ZOFF>(sp + g.own(b), spn);
            }
        }
        cs.hp[S1][b] = up[b];
    }
    if (REC && rec)
        record_add<(sizeof(R) == 8 ? 1 : BT)>(tc, acc);
    if constexpr (MEASURE) {
        // S(q + 1) went into the third plane at the start of the step
        __syncthreads();   // S(q + 1) complete; every thread is done with S(q - 1)
        return;
    }
    __syncthreads();   // S'(q - 1) complete; every thread is done with S(q) and S(q - 1)
    // S(q + 1) into the other S plane
    copy_next(nxt);
    if (g.interior) {
        const int zc = q - 2;
        const bool zc_own = zc >= z0 && zc < z1 && (zper || (zc >= 0 && zc < nz));
        // D: links from S'(q - 1) into planes q - 2 (completing it), q - 1 and
        // q (when S'(q - 1) does not exist, no site has links to it)
        V3<R> down[NB];   // plane q's first sums, moved into the slot of q - 2 after E
#pragma unroll
        for (int b = 0; b < NB; ++b)
            down[b] = V3<R>{0, 0, 0};
        if (zp_need) {
            if constexpr (KIND != kKindGeneric) {
                plane_links<R, KIND, NB, ZOFF>(sp, g, kj, cs.hc[S0], cs.hc[S1], down);
            } else {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    add_dz<R, KIND, NB, 1, ZOFF>(cs.hc[S0][b], sp, g, b, kj, pat, ent, plane_pattern(r, zc, b));
                    add_dz<R, KIND, NB, 0, ZOFF>(cs.hc[S1][b], sp, g, b, kj, pat, ent, plane_pattern(r, zp, b));
                    add_dz<R, KIND, NB, -1, ZOFF>(down[b], sp, g, b, kj, pat, ent, plane_pattern(r, q, b));
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            // E: corrector of plane q - 2
            if (zc_own) {
                const V3<R> s = cs.c_sp[S0][b];
                const R as = m.ani * dot(s, e);
                const V3<R> h{fma(as, e.x, cs.hc[S0][b].x) + cs.c_th[S0][b].x,
                              fma(as, e.y, cs.hc[S0][b].y) + cs.c_th[S0][b].y,
                              fma(as, e.z, cs.hc[S0][b].z) + cs.c_th[S0][b].z};
                // half the step's dS' dt (a step of dt / 2: the halving is exact)
                const V3<R> dsh = llg_step(s, h, (R)0.5 * r.gdt, r.alpha);
                const V3<R> sn = normalised(V3<R>{cs.c_base[S0][b].x + dsh.x, cs.c_base[S0][b].y + dsh.y,
                                                  cs.c_base[S0][b].z + dsh.z});
                // ordinary stores: the L2 merges the lanes' 12- or 24-byte
                // spins into whole lines (streaming stores of FP64 spins
                // reached memory as 1.4 times their bytes, for no gain in time)
                SLLG_GLOBAL R* dst =
                    (SLLG_GLOBAL R*)run.Sn + 3 * (int64_t)(g.col + (uint32_t)b + g.plane_sites * (uint32_t)zw_m2);
                dst[0] = sn.x;
                dst[1] = sn.y;
                dst[2] = sn.z;
                if (!spin_ok(sn))
                    flag_fault(r.fault);
            }
            cs.hc[S0][b] = down[b];
        }
    }
    __syncthreads();   // S(q + 1) complete; every thread is done with S'(q - 1)
}

template <typename R, int KIND, int NB, int BT, bool MEASURE, bool REC>
__device__ __forceinline__ void fused_item(const ReplicaDev<R>& r, const FusedItem& w, int k, char* lds,
                                           int plane_bytes, const int4* pat, const FEnt<R>* ent,
                                           double (*red)[BT / 64], double* acc_base, uint32_t* dcol)
{
    const int PX = r.f_px, PY = r.f_py, SW = PX + 2, SH = PY + 2, area = SW * SH;
    const int nx = r.f_nx, ny = r.f_ny, nz = r.f_nz;
    const bool zper = r.f_zper != 0;
    const int t = (int)threadIdx.x;
    ItemGeo<NB> g;
    g.live = t < PX * PY;
    // Threads of the tile first (row by row), then the ring (bottom row, top
    // row, left column, right column): the waves of the ring alone skip the
    // corrector phases as a whole.
    const int TX = PX - 2, inner = TX * (PY - 2);
    int px = 0, py = 0;
    if (t < inner) {
        py = 1 + t / TX;
        px = 1 + t - (py - 1) * TX;
    } else if (g.live) {
        int k = t - inner;
        if (k < 2 * PX) {
            py = k < PX ? 0 : PY - 1;
            px = k < PX ? k : k - PX;
        } else {
            k -= 2 * PX;
            px = k < PY - 2 ? 0 : PX - 1;
            py = 1 + (k < PY - 2 ? k : k - (PY - 2));
        }
    }
    const int ux = w.x0 - 1 + px, uy = w.y0 - 1 + py;   // cell, before wrapping
    g.interior = t < inner && ux < nx && uy < ny;
    g.col = (uint32_t)NB * (uint32_t)(wrap_cell(ux, nx) + nx * wrap_cell(uy, ny));
    g.plane_sites = (uint32_t)NB * (uint32_t)nx * (uint32_t)ny;
    constexpr int RW = PlaneLayout<R, BT>::RW, CPW = PlaneLayout<R, BT>::CPW;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
            g.rb[b][dy + 1] = (sizeof(R) == 4 ? b * area + (py + 1 + dy) * SW + px
                                              : (b * SH + py + 1 + dy) * 2 * RW + px) * 16;

    ItemRun<R> run;
    // the 16 bytes of S each lane copies per chunk of a plane (64 lanes, 1
    // KiB of LDS), kept in LDS.  FP32: LDS slot s = site (b, ry, rx) of the
    // region.  FP64: lane l of a chunk fills row c * 64 / (2 RW) + l / (2 RW)
    // (basis-major), site rx = l mod RW, x and y (first half of the row) or
    // z (second half, from 16 bytes into the site).
    run.n_chunks = fused_plane_chunks(PX, PY, NB, sizeof(R), BT);
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int c = (t >> 6) + j * (BT / 64), l = t & 63;
        int b, ry, rx, part = 0;
        bool valid;
        if constexpr (sizeof(R) == 4) {
            const int s = c * 64 + l;
            b = s / area;
            const int cell = s - b * area;
            ry = cell / SW;
            rx = cell - ry * SW;
            valid = s < area * NB;
        } else {
            const int row = c * (32 / RW) + l / (2 * RW);
            part = (l / RW) & 1;
            rx = l % RW;
            b = row / SH;
            ry = row - b * SH;
            valid = row < NB * SH && rx < SW;
        }
        const uint32_t site = (uint32_t)NB * (uint32_t)(wrap_cell(w.x0 - 2 + rx, nx) + nx * wrap_cell(w.y0 - 2 + ry, ny)) +
                              (uint32_t)b;
        dcol[j * BT + t] = valid ? site * 3u * (uint32_t)sizeof(R) + 16u * (uint32_t)part : 0xFFFFFFFFu;
    }
    run.dcol = dcol;
    // the measuring launch reads the state after the chunk's nsteps steps,
    // or with k < 0 the current state in place (Monte Carlo records)
    const int mslot = MEASURE ? (k < 0 ? 0 : r.nsteps) : k;
    const int par = (r.parity + mslot) & 1;
    run.S = r.S[par];
    run.Sn = r.S[par ^ 1];
    // the spin buffer holds 16 bytes past its last site (the copies read 16 bytes per lane)
    run.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<R*>(run.S), 0,
                                                 (int)(3u * (uint32_t)sizeof(R) * (uint32_t)r.n + 16u), 0x00020000);
    run.z0 = w.z0;
    run.z1 = w.z1;
    run.partials = REC && (r.flags & kRecord) && (MEASURE || k >= 1);
    run.step = r.step + (uint64_t)k;
    char* planes[2] = {lds, lds + plane_bytes};
    char* sp = lds + 2 * plane_bytes;
    // the thread's FP64 m and E sums: FP32 in LDS, FP64 in registers
    constexpr int AS = sizeof(R) == 8 ? 1 : BT;
    double acc_reg[4];
    double* acc;
    if constexpr (sizeof(R) == 8)
        acc = acc_reg;
    else
        acc = acc_base + t;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        acc[c * AS] = 0.0;

    const MaterialDev<R> m = uniform_material(r);
    ColumnState<R, NB> cs;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int b = 0; b < NB; ++b)
            cs.hp[i][b] = cs.hc[i][b] = cs.c_sp[i][b] = cs.c_base[i][b] = cs.c_th[i][b] = V3<R>{0, 0, 0};

    const int z0 = w.z0, z1 = w.z1;
    // wrapped plane numbers of q - 2, q - 1, q and q + 1, advanced by one per plane
    auto wrapz = [&](int z) { return zper ? wrap_cell(z, nz) : z; };
    int zw_m2 = wrapz(z0 - 4), zw_m1 = wrapz(z0 - 3), zw_0 = wrapz(z0 - 2), zw_p1 = wrapz(z0 - 1);
    {
        // S(z0 - 2) into plane 0
        const bool exists = zper || (z0 - 2 >= 0 && z0 - 2 < nz);
        const int wave = t >> 6, lane = t & 63;
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int c = wave + j * (BT / 64);
            if (c >= run.n_chunks)
                break;
            char* d = planes[0] + c * 64 * 16 + lane * 16;
            const uint32_t dc = dcol[j * BT + t];
            if (dc != 0xFFFFFFFFu) {
                if (exists) {
                    const R* src = reinterpret_cast<const R*>(reinterpret_cast<const char*>(run.S) + dc) +
                                   3 * (size_t)g.plane_sites * (uint32_t)zw_0;
                    if constexpr (sizeof(R) == 4)
                        *reinterpret_cast<Slot4*>(d) = Slot4{src[0], src[1], src[2], 0.0f};
                    else
                        *reinterpret_cast<XY64*>(d) = XY64{src[0], src[1]};
                } else {
                    *reinterpret_cast<Zero16*>(d) = Zero16{{0u, 0u, 0u, 0u}};
                }
            }
        }
    }
    __syncthreads();
    auto next_plane = [&] {
        zw_m2 = zw_m1;
        zw_m1 = zw_0;
        zw_0 = zw_p1;
        zw_p1 = zper ? (zw_p1 + 1 == nz ? 0 : zw_p1 + 1) : zw_p1 + 1;
    };
    if constexpr (MEASURE) {
        // three S planes in turn: S(q), S(q - 1), and the one S(q + 1) goes to
        char* cur = planes[0];
        char* prev = sp;   // S(z0 - 3): never read
        char* free_plane = planes[1];
        auto rotate = [&] {
            char* t = prev;
            prev = cur;
            cur = free_plane;
            free_plane = t;
        };
        for (int q = z0 - 2; q <= z1 + 1; q += 2) {
            plane_step<R, KIND, NB, BT, MEASURE, 0, REC>(r, g, run, cs, cur, prev, free_plane, acc, pat, ent, q, zw_m2,
                                                    zw_m1, zw_p1, m);
            rotate();
            next_plane();
            if (q + 1 > z1 + 1)
                break;
            plane_step<R, KIND, NB, BT, MEASURE, 1, REC>(r, g, run, cs, cur, prev, free_plane, acc, pat, ent, q + 1,
                                                    zw_m2, zw_m1, zw_p1, m);
            rotate();
            next_plane();
        }
    } else {
        for (int q = z0 - 2; q <= z1 + 1; q += 2) {
            plane_step<R, KIND, NB, BT, MEASURE, 0, REC>(r, g, run, cs, planes[0], planes[1], sp, acc, pat, ent, q, zw_m2,
                                                    zw_m1, zw_p1, m);
            next_plane();
            if (q + 1 > z1 + 1)
                break;
            plane_step<R, KIND, NB, BT, MEASURE, 1, REC>(r, g, run, cs, planes[1], planes[0], sp, acc, pat, ent, q + 1,
                                                    zw_m2, zw_m1, zw_p1, m);
            next_plane();
        }
    }
    if (run.partials) {
        const int lane = t & 63, wave = t >> 6;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double s = wave_sum(acc[c * AS]);
            if (lane == 0)
                red[c][wave] = s;
        }
        __syncthreads();
        if (t == 0) {
            double* out = r.f_partials + 4 * ((int64_t)(mslot & 1) * r.f_items + w.idx);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int q = 0; q < BT / 64; ++q)
                    s += red[c][q];
                out[c] = s;
            }
        }
    }
}

// One Heun step (k of the chunk) of every item, or with MEASURE the m and E
// sums of the current state of every recording replica.  Dynamic LDS: two
// S planes and one S' plane of plane_bytes each, then (generic kind) the
// pattern tables.
// Registers capped for four waves per SIMD in FP32 (two 512-lane or four
// 256-lane workgroups per compute unit), two in FP64 (twice the registers
// per column).
#ifndef SLLG_FUSED_WAVES
#define SLLG_FUSED_WAVES 4
#endif
#ifndef SLLG_FUSED_WAVES_F64
#define SLLG_FUSED_WAVES_F64 2
#endif

template <typename R, int KIND, int NB, int BT, bool MEASURE, bool REC>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? SLLG_FUSED_WAVES
                                                                                   : SLLG_FUSED_WAVES_F64))) void k_fused(const ReplicaDev<R>* __restrict__ reps,
                                              const FusedItem* __restrict__ items,
                                              const int* __restrict__ n_items, int k, int remap, int plane_bytes)
{
    // dynamic: two S planes, one S' plane, then (generic kind) the pattern
    // tables; static: the threads' FP64 m and E sums and the copy table,
    // separate objects so that their accesses need not wait for the plane
    // copies in flight
    extern __shared__ __attribute__((aligned(16))) char fused_lds[];
    __shared__ double red[4][BT / 64];
    __shared__ double acc[sizeof(R) == 8 ? 1 : 4 * BT];   // FP64 keeps these sums in registers
    __shared__ uint32_t dcol[PlaneLayout<R, BT>::CPW * BT];
    int4* pat = reinterpret_cast<int4*>(fused_lds + 3 * plane_bytes);
    FEnt<R>* ent = reinterpret_cast<FEnt<R>*>(pat + kFusedMaxPatterns);
    const int W = *n_items;
    int staged = -1;
    for (TileIter it(W, remap); it.more(); it.next()) {
        const FusedItem w = items[it.t];
        const ReplicaDev<R>& r = reps[w.replica];
        if (MEASURE ? (!(r.flags & kRecord) || r.nsteps <= 0) : k >= r.nsteps)
            continue;   // uniform over the block
        __syncthreads();   // every thread is done with the previous item's LDS
        if (KIND == kKindGeneric && w.replica != staged) {
            for (int q = (int)threadIdx.x; q < r.f_npat; q += BT)
                pat[q] = reinterpret_cast<const int4*>(r.f_pat)[q];
            for (int q = (int)threadIdx.x; q < r.f_nent; q += BT)
                ent[q] = reinterpret_cast<const FEnt<R>*>(r.f_ent)[q];
            staged = w.replica;
            __syncthreads();
        }
        // items' sums of the previous launch -> the record two steps back
        if (REC && !MEASURE && w.idx == 0 && (r.flags & kRecord) && k >= 2)
            fused_record<R, BT>(r, (k - 1) & 1, k - 2, red);
        fused_item<R, KIND, NB, BT, MEASURE, REC>(r, w, k, fused_lds, plane_bytes, pat, ent, red, acc, dcol);
    }
}

// After the measuring launch, one workgroup per replica: the last two
// records of the chunk, the averaging sums of its records, then the step
// counter, parity and record position advance (one launch for the chunk's
// end instead of three).
template <typename R>
__global__ __launch_bounds__(256) void k_fused_finish(ReplicaDev<R>* __restrict__ reps)
{
    __shared__ double red[4][4];
    ReplicaDev<R>& r = reps[blockIdx.x];
    if (r.nsteps <= 0)
        return;   // uniform over the block
    if ((r.flags & kFused) && (r.flags & kRecord)) {
        if (r.nsteps >= 2)
            fused_record<R, 256>(r, (r.nsteps - 1) & 1, r.nsteps - 2, red);
        fused_record<R, 256>(r, r.nsteps & 1, r.nsteps - 1, red);
    }
    // thread 0 wrote the records (fused_record) and reads them back here
    if (threadIdx.x == 0) {
        accumulate_records(r);
        advance_replica(r);
    }
}

// After a measuring launch of the current state (k < 0), one workgroup per
// replica: the items' sums into record `slot` (Monte Carlo records; no
// advance of the step counter or parity).
template <typename R>
__global__ __launch_bounds__(256) void k_fused_record(ReplicaDev<R>* __restrict__ reps, int slot)
{
    __shared__ double red[4][4];
    const ReplicaDev<R>& r = reps[blockIdx.x];
    if (r.nsteps <= 0 || !(r.flags & kFused) || !(r.flags & kRecord))
        return;   // uniform over the block
    fused_record<R, 256>(r, 0, slot, red);
}

// The measuring launch always records; a step launch records unless no
// replica of the batch takes records (rec false: the variant without the
// record code).
template <typename R, int KIND, int NB, int BT>
const void* fused_ptr(bool measure, bool rec)
{
    if (measure)
        return (const void*)k_fused<R, KIND, NB, BT, true, true>;
    return rec ? (const void*)k_fused<R, KIND, NB, BT, false, true> : (const void*)k_fused<R, KIND, NB, BT, false, false>;
}

// The kernel of (kind, nb, bt, measure), or null if it is not built
// (FP64: the compiled kinds, 256 and 512 threads).
template <typename R>
const void* fused_kernel(int kind, int nb, int bt, bool measure, bool rec = true)
{
#define SLLG_FUSED_CASE(K_, NB_, BT_)           \
    if (kind == K_ && nb == NB_ && bt == BT_)   \
        return fused_ptr<R, K_, NB_, BT_>(measure, rec);
    SLLG_FUSED_CASE(kKindSc6, 1, 256)
    SLLG_FUSED_CASE(kKindSc6, 1, 512)
    SLLG_FUSED_CASE(kKindBcc8, 2, 256)
    SLLG_FUSED_CASE(kKindBcc8, 2, 512)
    SLLG_FUSED_CASE(kKindBcc14, 2, 256)
    SLLG_FUSED_CASE(kKindBcc14, 2, 512)
    if constexpr (sizeof(R) == 4) {
        SLLG_FUSED_CASE(kKindSc6, 1, 1024)
        SLLG_FUSED_CASE(kKindBcc8, 2, 1024)
        SLLG_FUSED_CASE(kKindBcc14, 2, 1024)
        SLLG_FUSED_CASE(kKindGeneric, 1, 256)
        SLLG_FUSED_CASE(kKindGeneric, 1, 512)
        SLLG_FUSED_CASE(kKindGeneric, 2, 256)
        SLLG_FUSED_CASE(kKindGeneric, 2, 512)
    }
#undef SLLG_FUSED_CASE
    return nullptr;
}

}  // namespace

bool fused_block_ok(int kind, int bt, size_t real_bytes)
{
    if (real_bytes == 4)
        return bt == 256 || bt == 512 || (bt == 1024 && kind != kKindGeneric);
    return (bt == 256 || bt == 512) && kind != kKindGeneric;
}

size_t fused_static_lds(int bt, size_t real_bytes)
{
    // acc (FP32 only), dcol and red of k_fused
    const size_t acc = real_bytes == 8 ? sizeof(double) : (size_t)bt * 4 * sizeof(double);
    return acc + (size_t)bt * (size_t)fused_chunks_per_wave(real_bytes) * sizeof(uint32_t) +
           4 * (size_t)(bt / 64) * sizeof(double);
}

size_t fused_lds_bytes(int kind, int plane_bytes, int bt)
{
    // dynamic part only; the static arrays come on top (fused_static_lds)
    (void)bt;
    size_t b = 3 * (size_t)plane_bytes;
    if (kind == kKindGeneric)
        b += kFusedMaxPatterns * sizeof(int4) + kFusedMaxEntries * sizeof(FusedEntryD);
    return b;
}

template <typename R>
hipError_t launch_fused(const ReplicaDev<R>* reps, const FusedItem* items, const int* n_items, int grid, int k,
                        int remap, bool measure, bool rec, int kind, int nb, int bt, int plane_bytes, hipStream_t st)
{
    if (grid <= 0)
        return hipSuccess;
    const void* f = fused_kernel<R>(kind, nb, bt, measure, rec);
    if (!f)
        return hipErrorInvalidValue;
    void* args[] = {(void*)&reps, (void*)&items, (void*)&n_items, (void*)&k, (void*)&remap, (void*)&plane_bytes};
    return hipLaunchKernel(f, dim3(grid), dim3(bt), args, fused_lds_bytes(kind, plane_bytes, bt), st);
}

template <typename R>
hipError_t launch_fused_finish(ReplicaDev<R>* reps, int n_rep, hipStream_t st)
{
    if (n_rep <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_fused_finish<R>), dim3(n_rep), dim3(256), 0, st, reps);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fused_record(ReplicaDev<R>* reps, int n_rep, int slot, hipStream_t st)
{
    if (n_rep <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_fused_record<R>), dim3(n_rep), dim3(256), 0, st, reps, slot);
    return hipGetLastError();
}

template <typename R>
int fused_resident_blocks(int device, int kind, int nb, int bt, int plane_bytes)
{
    int cus = 0, a = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        return 0;
    const void* f = fused_kernel<R>(kind, nb, bt, false);
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, f, bt, fused_lds_bytes(kind, plane_bytes, bt)) !=
                  hipSuccess)
        return 0;
    return cus * a;
}

// LDS one workgroup may take (the device limit).
size_t fused_lds_limit(int device)
{
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || v <= 0)
        return 64 * 1024;
    return (size_t)v;
}

template hipError_t launch_fused<float>(const ReplicaDev<float>*, const FusedItem*, const int*, int, int, int, bool,
                                        bool, int, int, int, int, hipStream_t);
template hipError_t launch_fused<double>(const ReplicaDev<double>*, const FusedItem*, const int*, int, int, int, bool,
                                         bool, int, int, int, int, hipStream_t);
template hipError_t launch_fused_finish<float>(ReplicaDev<float>*, int, hipStream_t);
template hipError_t launch_fused_finish<double>(ReplicaDev<double>*, int, hipStream_t);
template hipError_t launch_fused_record<float>(ReplicaDev<float>*, int, int, hipStream_t);
template hipError_t launch_fused_record<double>(ReplicaDev<double>*, int, int, hipStream_t);
template int fused_resident_blocks<float>(int, int, int, int, int);
template int fused_resident_blocks<double>(int, int, int, int, int);

}  // namespace sllg
