// Device helpers shared by the step kernels (kernels.hip) and the fused
// plane-marching step (fused.hip): the counter-based noise, the LLG
// right-hand side, vector helpers, work distribution over workgroups and
// the fixed-order wavefront sums of the FP64 reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.hpp"

// Streaming (non-temporal) stores of S' and S, and the corrector's loads of
// the old S (read once): measured faster on MI355X for the loads, and for
// FP64 stores.
#ifndef SLLG_NT_STORES_F32
#define SLLG_NT_STORES_F32 0
#endif
#ifndef SLLG_NT_STORES_F64
#define SLLG_NT_STORES_F64 1
#endif
#ifndef SLLG_NT_LOADS
#define SLLG_NT_LOADS 1
#endif

namespace sllg {
namespace dev {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products; the key is bumped by the Weyl constants between
// rounds.
// ---------------------------------------------------------------------------
// a ^ b ^ c in one instruction: the three-input bitwise operation of gfx950
// with truth table 0x96 (set where an odd number of inputs is set).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // the first two rounds still mix counter words that are the same
        // across the wavefront (step and purpose), which stay on the scalar
        // unit with plain xors
        const uint32_t n0 = r < 2 ? (uint32_t)(p1 >> 32) ^ c1 ^ k0 : xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = r < 2 ? (uint32_t)(p0 >> 32) ^ c3 ^ k1 : xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Three standard normals for (site, step): counter (site, step lo, step hi,
// purpose), key = seed (purpose 0: the thermal field, 2: Monte Carlo trial
// moves); Box-Muller on the pairs (r0, r1) and (r2, r3), the fourth normal
// dropped.  Uniforms u = (r + 1) 2^-32 in (0, 1] for the radius,
// u' = r 2^-32 in [0, 1) for the angle.
__device__ __forceinline__ void thermal_normals(uint64_t seed, uint64_t step, uint32_t site,
                                                float g[3], uint32_t purpose = 0u)
{
    uint32_t c0 = site, c1 = (uint32_t)step, c2 = (uint32_t)(step >> 32), c3 = purpose;
    philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float two_m32 = 2.3283064365386963e-10f;   // 2^-32
    const float u1 = ((float)c0 + 1.0f) * two_m32;
    const float u3 = ((float)c2 + 1.0f) * two_m32;
    const float a2 = (float)c1 * two_m32;             // angle in revolutions
    const float a4 = (float)c3 * two_m32;
    // -2 ln u = -2 ln(2) log2(u); v_log_f32 is log2, v_sin/v_cos take revolutions
    const float rho1 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    const float rho2 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u3));
    g[0] = rho1 * __builtin_amdgcn_cosf(a2);
    g[1] = rho1 * __builtin_amdgcn_sinf(a2);
    g[2] = rho2 * __builtin_amdgcn_cosf(a4);
}

// FP64 natural logarithm of u in (0, 1] (no zero, infinity or NaN
// arrives).  u = m 2^e with m in [sqrt(1/2), sqrt(2)); f = m - 1 is exact;
// with s = f / (2 + f), log m = 2 atanh(s) = f - s (f - R), R = sum over
// k >= 1 of 2 s^(2k) / (2k + 1): |s| <= 0.1716, so ten terms leave a
// truncation error below 2^-60 of the result.  s comes from a hardware
// reciprocal refined by two Newton steps and one residual correction; e ln 2
// is added with ln 2 as a double plus its rounding error.
__device__ __forceinline__ double log_unit(double u)
{
    double m = __builtin_amdgcn_frexp_mant(u);   // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(u);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;
    const double d = 2.0 + f;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    double s = f * r;
    s = fma(fma(-s, d, f), r, s);
    const double z = s * s;
    double p = 2.0 / 21.0;
    p = fma(p, z, 2.0 / 19.0);
    p = fma(p, z, 2.0 / 17.0);
    p = fma(p, z, 2.0 / 15.0);
    p = fma(p, z, 2.0 / 13.0);
    p = fma(p, z, 2.0 / 11.0);
    p = fma(p, z, 2.0 / 9.0);
    p = fma(p, z, 2.0 / 7.0);
    p = fma(p, z, 2.0 / 5.0);
    p = fma(p, z, 2.0 / 3.0);
    const double logm = fma(-s, fma(-z, p, f), f);
    const double ln2 = 0.6931471805599453;        // ln 2 rounded to double
    const double ln2_err = 2.3190468138462996e-17;   // ln 2 minus that double
    const double ed = (double)e;
    return fma(ed, ln2, fma(ed, ln2_err, logm));
}

// cos and sin of 2 pi a for the angle a = c 2^-32 revolutions.  The nearest
// quarter turn j = round(4 a) (mod 4) and the rest r = a - j/4 in [-1/8, 1/8)
// come exactly from the integer; x = 2 pi r, |x| <= pi/4, and the Taylor
// series of sin x to x^17 and of cos x to x^18 (later terms below 2^-56
// relative); then the quarter turn swaps and negates them.
__device__ __forceinline__ void cossin_turns(uint32_t c, double& cs, double& sn)
{
    const uint32_t j = (c + 0x20000000u) >> 30;
    const int32_t ri = (int32_t)(c - (j << 30));
    const double x = (double)ri * (6.283185307179586 * 2.3283064365386963e-10);
    const double z = x * x;
    double ps = -1.0 / 355687428096000.0;          // -1/17!
    ps = fma(ps, z, 1.0 / 1307674368000.0);        //  1/15!
    ps = fma(ps, z, -1.0 / 6227020800.0);          // -1/13!
    ps = fma(ps, z, 1.0 / 39916800.0);             //  1/11!
    ps = fma(ps, z, -1.0 / 362880.0);              // -1/9!
    ps = fma(ps, z, 1.0 / 5040.0);                 //  1/7!
    ps = fma(ps, z, -1.0 / 120.0);                 // -1/5!
    ps = fma(ps, z, 1.0 / 6.0);
    const double sx = fma(-x * z, ps, x);          // x - x^3 (1/3! - ...)
    double pc = 1.0 / 6402373705728000.0;          //  1/18!
    pc = fma(pc, z, -1.0 / 20922789888000.0);      // -1/16!
    pc = fma(pc, z, 1.0 / 87178291200.0);          //  1/14!
    pc = fma(pc, z, -1.0 / 479001600.0);           // -1/12!
    pc = fma(pc, z, 1.0 / 3628800.0);              //  1/10!
    pc = fma(pc, z, -1.0 / 40320.0);               // -1/8!
    pc = fma(pc, z, 1.0 / 720.0);                  //  1/6!
    pc = fma(pc, z, -1.0 / 24.0);                  // -1/4!
    const double cx = fma(z * z, -pc, fma(-0.5, z, 1.0));   // 1 - x^2/2 + x^4 (1/4! - ...)
    const bool swap = j & 1u;
    const double c0 = swap ? sx : cx, s0 = swap ? cx : sx;
    cs = ((j + 1u) & 2u) ? -c0 : c0;
    sn = (j & 2u) ? -s0 : s0;
}

// sqrt(v) for v >= 0 (a zero gives zero): the hardware reciprocal square
// root estimate y, one Goldschmidt step for g ~ sqrt(v) and h ~ 1/(2 sqrt v)
// from g = v y, h = y/2, then two residual corrections g += (v - g^2) h.
__device__ __forceinline__ double sqrt_nonneg(double v)
{
    const double y = __builtin_amdgcn_rsq(v);
    double g = v * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    g = fma(fma(-g, g, v), h, g);
    g = fma(fma(-g, g, v), h, g);
    return v > 0.0 ? g : 0.0;
}

__device__ __forceinline__ void thermal_normals(uint64_t seed, uint64_t step, uint32_t site,
                                                double g[3], uint32_t purpose = 0u)
{
    uint32_t c0 = site, c1 = (uint32_t)step, c2 = (uint32_t)(step >> 32), c3 = purpose;
    philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double two_m32 = 2.3283064365386963e-10;
    const double u1 = ((double)c0 + 1.0) * two_m32;
    const double u3 = ((double)c2 + 1.0) * two_m32;
    const double rho1 = sqrt_nonneg(-2.0 * log_unit(u1));
    const double rho2 = sqrt_nonneg(-2.0 * log_unit(u3));
    double cs2, sn2, cs4, sn4;
    cossin_turns(c1, cs2, sn2);
    cossin_turns(c3, cs4, sn4);
    (void)sn4;
    g[0] = rho1 * cs2;
    g[1] = rho1 * sn2;
    g[2] = rho2 * cs4;
}

__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
// 1/sqrt(x) for x > 0 (a spin's squared norm after a step, close to 1): the
// hardware estimate refined by two Newton steps y <- y + (y/2)(1 - x y^2).
__device__ __forceinline__ double rsqrt_r(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return y;
}

template <typename R>
struct V3 {
    R x, y, z;
};

// Every buffer the kernels touch lives in global memory; saying so lets the
// compiler emit global_load/global_store instead of generic flat accesses
// for pointers it reads out of the replica table.
#define SLLG_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ T gload(const T* p, int64_t i)
{
    return ((const SLLG_GLOBAL T*)p)[i];
}

template <typename R>
__device__ __forceinline__ V3<R> load3(const R* __restrict__ p, int64_t i)
{
    const SLLG_GLOBAL R* g = (const SLLG_GLOBAL R*)p + 3 * i;
    return V3<R>{g[0], g[1], g[2]};
}

template <typename R>
__device__ __forceinline__ void store3(R* __restrict__ p, int64_t i, V3<R> v)
{
    SLLG_GLOBAL R* g = (SLLG_GLOBAL R*)p + 3 * i;
    if constexpr (sizeof(R) == 4 ? SLLG_NT_STORES_F32 : SLLG_NT_STORES_F64) {
        __builtin_nontemporal_store(v.x, &g[0]);
        __builtin_nontemporal_store(v.y, &g[1]);
        __builtin_nontemporal_store(v.z, &g[2]);
    } else {
        g[0] = v.x;
        g[1] = v.y;
        g[2] = v.z;
    }
}

// The corrector's own old spin: read once, so streamed past the caches when
// enabled.
template <typename R>
__device__ __forceinline__ V3<R> load3_once(const R* __restrict__ p, int64_t i)
{
    const SLLG_GLOBAL R* g = (const SLLG_GLOBAL R*)p + 3 * i;
#if SLLG_NT_LOADS
    return V3<R>{__builtin_nontemporal_load(&g[0]), __builtin_nontemporal_load(&g[1]),
                 __builtin_nontemporal_load(&g[2])};
#else
    return V3<R>{g[0], g[1], g[2]};
#endif
}

template <typename R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z;
}

// dS dt = -gamma dt/(1+lambda^2) [S x H + lambda S x (S x H)]
template <typename R>
__device__ __forceinline__ V3<R> llg_step(V3<R> s, V3<R> h, R gdt, R alpha)
{
    const V3<R> a{s.y * h.z - s.z * h.y, s.z * h.x - s.x * h.z, s.x * h.y - s.y * h.x};
    const V3<R> b{s.y * a.z - s.z * a.y, s.z * a.x - s.x * a.z, s.x * a.y - s.y * a.x};
    return V3<R>{-gdt * (a.x + alpha * b.x), -gdt * (a.y + alpha * b.y), -gdt * (a.z + alpha * b.z)};
}

// Whether a new spin is usable: a unit vector has |x| + |y| + |z| <= sqrt 3,
// a NaN or infinite component fails the comparison.
template <typename R>
__device__ __forceinline__ bool spin_ok(const V3<R>& s)
{
    return fabs(s.x) + fabs(s.y) + fabs(s.z) <= (R)2;
}

// Flags a non-finite spin for the host (a plain store: every writer stores 1).
__device__ __forceinline__ void flag_fault(int32_t* fault)
{
    *(volatile int32_t*)fault = 1;
}

template <typename R>
__device__ __forceinline__ V3<R> normalised(V3<R> v)
{
    const R inv = rsqrt_r(dot(v, v));
    return V3<R>{v.x * inv, v.y * inv, v.z * inv};
}


// Work distribution.  A launch has a fixed number of workgroups (about the
// number that fit on the chip at once), each sweeping many tiles.
// Workgroups are handed to the 8 XCDs round-robin.  Mode 0: plain
// grid-stride.  Mode 1: the workgroups of XCD x share one contiguous range
// of tiles (neighbouring sites meet in that XCD's L2), interleaved tile by
// tile.  Mode 2: the same XCD ranges, each split into one contiguous run of
// tiles per workgroup (the previous tiles of a run are still in the
// workgroup's L1 when the next one needs them).
struct TileIter {
    int64_t t, end, stride;
    __device__ TileIter(int W, int mode)
    {
        const int G = (int)gridDim.x, b = (int)blockIdx.x;
        if (mode != 0 && (G & 7) == 0) {
            const int x = b & 7, u = b >> 3, Gx = G >> 3;
            const int64_t lo = (int64_t)W * x / 8, hi = (int64_t)W * (x + 1) / 8;
            if (mode == 2) {
                const int64_t run = (hi - lo + Gx - 1) / Gx;
                t = lo + (int64_t)u * run;
                end = t + run < hi ? t + run : hi;
                stride = 1;
            } else {
                t = lo + u;
                end = hi;
                stride = Gx;
            }
        } else {
            t = b;
            end = W;
            stride = G;
        }
    }
    __device__ bool more() const { return t < end; }
    __device__ void next() { t += stride; }
};

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const uint64_t u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sum within each row of 16 lanes (quad swaps, then rotations by 4 and 8).
template <typename T>
__device__ __forceinline__ T row_sum(T v)
{
    if constexpr (sizeof(T) == 4) {
        v += dpp_f<0xB1>(v);    // quad_perm [1,0,3,2]
        v += dpp_f<0x4E>(v);    // quad_perm [2,3,0,1]
        v += dpp_f<0x124>(v);   // row_ror:4
        v += dpp_f<0x128>(v);   // row_ror:8
    } else {
        v += dpp_d<0xB1>(v);
        v += dpp_d<0x4E>(v);
        v += dpp_d<0x124>(v);
        v += dpp_d<0x128>(v);
    }
    return v;
}

__device__ __forceinline__ double lane_value(double v, int lane)
{
    const uint64_t u = __double_as_longlong(v);
    const uint32_t l = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)h << 32) | l));
}

__device__ __forceinline__ double lane_value(float v, int lane)
{
    return (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Wavefront total: rows of 16 lanes, then the four rows.
__device__ __forceinline__ double wave_sum(double v)
{
    v = row_sum(v);
    return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}


// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ float wave_uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double wave_uniform(double v)
{
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}


// The replica's only material (no per-site materials), in scalar registers.
template <typename R>
__device__ __forceinline__ MaterialDev<R> uniform_material(const ReplicaDev<R>& r)
{
    const SLLG_GLOBAL MaterialDev<R>& g = *(const SLLG_GLOBAL MaterialDev<R>*)r.mat;
    MaterialDev<R> m;
    m.mu_rel = wave_uniform(g.mu_rel);
    m.mu_frac = wave_uniform(g.mu_frac);
    m.ani = wave_uniform(g.ani);
    m.ku_mu = wave_uniform(g.ku_mu);
    m.sigma = wave_uniform(g.sigma);
    m.axis[0] = wave_uniform(g.axis[0]);
    m.axis[1] = wave_uniform(g.axis[1]);
    m.axis[2] = wave_uniform(g.axis[2]);
    m.cub = 0;     // cubic anisotropy takes the general variant
    m.kc_mu = 0;
    m.mu_s = wave_uniform(g.mu_s);
    return m;
}

// End of a chunk for one replica (one thread): the averaging block sums of
// the chunk's records (kAverage), then the step counter, buffer parity and
// record position advance by the chunk's steps.
template <typename R>
__device__ inline void accumulate_records(const ReplicaDev<R>& r)
{
    if (r.nsteps <= 0 || !(r.flags & kAverage))
        return;
    for (int t = 0; t < r.nsteps; ++t) {
        const int64_t sample = (int64_t)(r.step + (uint64_t)t) - r.avg_first;
        if (sample < 0)
            continue;
        const int64_t b = sample / r.avg_block_len;
        if (b >= r.avg_blocks)
            break;
        const double* rec = r.records + 4 * (r.rec_pos + t);
        const double mx = rec[0], my = rec[1], mz = rec[2];
        double* a = r.acc + 5 * b;
        a[0] += sqrt(mx * mx + my * my + mz * mz);
        a[1] += mx;
        a[2] += my;
        a[3] += mz;
        a[4] += rec[3];
    }
}

template <typename R>
__device__ inline void advance_replica(ReplicaDev<R>& r)
{
    const int ns = r.nsteps;
    if (ns > 0) {
        r.step += (uint64_t)ns;
        r.parity = (r.parity + ns) & 1;
        if (r.flags & kRecordSeries)
            r.rec_pos += ns;
    }
}

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

}  // namespace dev
}  // namespace sllg
