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
// site); neighbours are SELL-64 (a slice of 64 consecutive rows is stored
// column-major, so lane l of a wavefront reads entry k of its row at
// nb[slice_off + 64 k + l]: every load instruction of the gather is one
// contiguous 256-byte run); each entry packs type << 28 | column.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "layout.hpp"

namespace sllg {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products; the key is bumped by the Weyl constants between
// rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Three standard normals for (site, step): counter (site, step lo, step hi,
// 0), key = seed; Box-Muller on the pairs (r0, r1) and (r2, r3), the fourth
// normal dropped.  Uniforms u = (r + 1) 2^-32 in (0, 1] for the radius,
// u' = r 2^-32 in [0, 1) for the angle.
__device__ __forceinline__ void thermal_normals(uint64_t seed, uint64_t step, uint32_t site,
                                                float g[3])
{
    uint32_t c0 = site, c1 = (uint32_t)step, c2 = (uint32_t)(step >> 32), c3 = 0u;
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

__device__ __forceinline__ void thermal_normals(uint64_t seed, uint64_t step, uint32_t site,
                                                double g[3])
{
    uint32_t c0 = site, c1 = (uint32_t)step, c2 = (uint32_t)(step >> 32), c3 = 0u;
    philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double two_m32 = 2.3283064365386963e-10;
    const double u1 = ((double)c0 + 1.0) * two_m32;
    const double u3 = ((double)c2 + 1.0) * two_m32;
    const double rho1 = sqrt(-2.0 * log(u1));
    const double rho2 = sqrt(-2.0 * log(u3));
    double s2, c2d, s4, c4d;
    sincospi(2.0 * ((double)c1 * two_m32), &s2, &c2d);
    sincospi(2.0 * ((double)c3 * two_m32), &s4, &c4d);
    (void)s4;
    g[0] = rho1 * c2d;
    g[1] = rho1 * s2;
    g[2] = rho2 * c4d;
}

__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }

template <typename R>
struct V3 {
    R x, y, z;
};

template <typename R>
__device__ __forceinline__ V3<R> load3(const R* __restrict__ p, int64_t i)
{
    return V3<R>{p[3 * i], p[3 * i + 1], p[3 * i + 2]};
}

template <typename R>
__device__ __forceinline__ void store3(R* __restrict__ p, int64_t i, V3<R> v)
{
    p[3 * i] = v.x;
    p[3 * i + 1] = v.y;
    p[3 * i + 2] = v.z;
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

template <typename R>
__device__ __forceinline__ V3<R> normalised(V3<R> v)
{
    const R inv = rsqrt_r(dot(v, v));
    return V3<R>{v.x * inv, v.y * inv, v.z * inv};
}

// sum_k jt[type_k] S[col_k] over the SELL row of site i.
template <typename R>
__device__ __forceinline__ V3<R> exchange_sum(const ReplicaDev<R>& r, const R* __restrict__ S,
                                              const R* jt, int i)
{
    const int64_t base = r.slice_off[i >> 6] + (i & 63);
    const int d = r.deg[i];
    const uint32_t* __restrict__ p = r.nb + base;
    V3<R> h{0, 0, 0};
#pragma unroll 2
    for (int k = 0; k < d; ++k) {
        const uint32_t e = p[(int64_t)k * kSlice];
        const R J = jt[e >> kColBits];
        const V3<R> sj = load3(S, (int64_t)(e & kColMask));
        h.x += J * sj.x;
        h.y += J * sj.y;
        h.z += J * sj.z;
    }
    return h;
}

__device__ __forceinline__ int logical_block(int b, int n, int remap)
{
    if (!remap)
        return b;
    // Workgroups are handed to the 8 XCDs round-robin; give XCD x one
    // contiguous range of blocks so neighbouring sites share its L2.
    const int q = n >> 3, rem = n & 7;
    const int x = b & 7, idx = b >> 3;
    return x * q + (x < rem ? x : rem) + idx;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum of four doubles in a fixed order; result valid in thread 0.
__device__ __forceinline__ void block_sum4(double acc[4], double (*red)[kBlockSites / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double v = wave_sum(acc[c]);
        if (lane == 0)
            red[c][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int w = 0; w < kBlockSites / 64; ++w)
                s += red[c][w];
            acc[c] = s;
        }
    }
}

// Sum the per-block partials of one replica (fixed order, independent of the
// launch) into record `slot`: m = sum mu S / sum mu, and E.
template <typename R>
__device__ void finalize_record(const ReplicaDev<R>& r, int slot, double (*red)[kBlockSites / 64])
{
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < r.blocks; b += kBlockSites) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            acc[c] += r.partials[4 * (int64_t)b + c];
    }
    block_sum4(acc, red);
    if (threadIdx.x == 0) {
        double* out = r.records + 4 * (r.rec_pos + slot);
        out[0] = acc[0] * r.inv_mu_total;
        out[1] = acc[1] * r.inv_mu_total;
        out[2] = acc[2] * r.inv_mu_total;
        out[3] = acc[3];
    }
}

template <typename R>
__device__ __forceinline__ const MaterialDev<R>& site_material(const ReplicaDev<R>& r, int i)
{
    return (r.flags & kPerSiteMaterial) ? r.mat[r.matid[i]] : r.mat[0];
}

template <typename R>
__device__ __forceinline__ V3<R> site_axis(const ReplicaDev<R>& r, const MaterialDev<R>& m, int i)
{
    if (r.flags & kPerSiteAxis)
        return load3(r.axis, i);
    return V3<R>{m.axis[0], m.axis[1], m.axis[2]};
}

// ---------------------------------------------------------------------------
// Predictor.  For step k of the chunk: reads S (current state), writes the
// predicted spin S' = |S + dS dt| and the corrector base S + dS dt / 2.
// With MEASURE it only evaluates m and E of the state after the chunk.
// When recording, the energy and magnetisation of the current state (the
// state after the previous step) go to the replica's block partials: the
// exchange field needed for the energy is the one the predictor computes.
// ---------------------------------------------------------------------------
template <typename R, bool MEASURE>
__global__ __launch_bounds__(kBlockSites) void k_predict(const ReplicaDev<R>* __restrict__ reps,
                                                         const WorkItem* __restrict__ work,
                                                         const int* __restrict__ n_work, int k,
                                                         int remap)
{
    __shared__ R jt_s[kMaxTypes];
    __shared__ double red[4][kBlockSites / 64];
    const int lb = logical_block((int)blockIdx.x, (int)gridDim.x, remap);
    if (lb >= *n_work)
        return;
    const WorkItem w = work[lb];
    const ReplicaDev<R>& r = reps[w.replica];
    // MEASURE with k == 0: the state after this chunk's steps; k == 1: the
    // current state (no steps taken).
    const int nsteps = r.nsteps;
    if (MEASURE ? (!(r.flags & kRecord) || (k == 0 && nsteps <= 0)) : (k >= nsteps))
        return;   // uniform over the block
    const bool record = MEASURE || (r.flags & kRecord);
    if (threadIdx.x < kMaxTypes)
        jt_s[threadIdx.x] = r.jt[threadIdx.x];
    __syncthreads();

    const int i = w.block * kBlockSites + (int)threadIdx.x;
    const int par = (r.parity + (MEASURE ? (k == 0 ? nsteps : 0) : k)) & 1;
    const R* __restrict__ S = r.S[par];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < r.n) {
        const MaterialDev<R>& m = site_material(r, i);
        const V3<R> s = load3(S, i);
        const V3<R> sum = exchange_sum(r, S, jt_s, i);
        const V3<R> hex{m.mu_rel * sum.x, m.mu_rel * sum.y, m.mu_rel * sum.z};
        const V3<R> e = site_axis(r, m, i);
        const R se = dot(s, e);
        const V3<R> Happ{r.H[0], r.H[1], r.H[2]};
        if (record) {
            const double mu = m.mu_s;
            acc[0] = mu * (double)s.x;
            acc[1] = mu * (double)s.y;
            acc[2] = mu * (double)s.z;
            const R eu = (R)0.5 * dot(s, hex) + m.ku_mu * se * se + dot(s, Happ);
            acc[3] = -mu * (double)eu;
        }
        if (!MEASURE) {
            V3<R> h{hex.x + m.ani * se * e.x + Happ.x, hex.y + m.ani * se * e.y + Happ.y,
                    hex.z + m.ani * se * e.z + Happ.z};
            if (m.sigma != (R)0) {
                R g[3];
                thermal_normals(r.seed, r.step + (uint64_t)k, (uint32_t)i, g);
                h.x += m.sigma * g[0];
                h.y += m.sigma * g[1];
                h.z += m.sigma * g[2];
            }
            const V3<R> ds = llg_step(s, h, r.gdt, r.alpha);
            const V3<R> sp = normalised(V3<R>{s.x + ds.x, s.y + ds.y, s.z + ds.z});
            store3(r.Sp, i, sp);
            store3(r.Bc, i, V3<R>{s.x + (R)0.5 * ds.x, s.y + (R)0.5 * ds.y, s.z + (R)0.5 * ds.z});
        }
    }
    if (record) {
        block_sum4(acc, red);
        if (threadIdx.x == 0) {
            double* p = r.partials + 4 * (int64_t)w.block;
            p[0] = acc[0];
            p[1] = acc[1];
            p[2] = acc[2];
            p[3] = acc[3];
        }
    }
}

// ---------------------------------------------------------------------------
// Corrector.  Field at S' with the same thermal numbers (same counter),
// slope dS', and S_new = |S + (dS + dS') dt / 2| written to the other
// ping-pong buffer.  Block 0 of each recording replica also reduces the
// partials the predictor of this step left (the state after step k - 1).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlockSites) void k_correct(const ReplicaDev<R>* __restrict__ reps,
                                                         const WorkItem* __restrict__ work,
                                                         const int* __restrict__ n_work, int k,
                                                         int remap)
{
    __shared__ R jt_s[kMaxTypes];
    __shared__ double red[4][kBlockSites / 64];
    const int lb = logical_block((int)blockIdx.x, (int)gridDim.x, remap);
    if (lb >= *n_work)
        return;
    const WorkItem w = work[lb];
    const ReplicaDev<R>& r = reps[w.replica];
    if (k >= r.nsteps)
        return;
    if (threadIdx.x < kMaxTypes)
        jt_s[threadIdx.x] = r.jt[threadIdx.x];
    __syncthreads();

    const int i = w.block * kBlockSites + (int)threadIdx.x;
    if (i < r.n) {
        const MaterialDev<R>& m = site_material(r, i);
        const V3<R> sp = load3((const R*)r.Sp, i);
        const V3<R> sum = exchange_sum(r, (const R*)r.Sp, jt_s, i);
        const V3<R> e = site_axis(r, m, i);
        const R se = dot(sp, e);
        V3<R> h{m.mu_rel * sum.x + m.ani * se * e.x + r.H[0],
                m.mu_rel * sum.y + m.ani * se * e.y + r.H[1],
                m.mu_rel * sum.z + m.ani * se * e.z + r.H[2]};
        if (m.sigma != (R)0) {
            R g[3];
            thermal_normals(r.seed, r.step + (uint64_t)k, (uint32_t)i, g);
            h.x += m.sigma * g[0];
            h.y += m.sigma * g[1];
            h.z += m.sigma * g[2];
        }
        const V3<R> ds = llg_step(sp, h, r.gdt, r.alpha);
        const V3<R> b = load3((const R*)r.Bc, i);
        const V3<R> sn = normalised(V3<R>{b.x + (R)0.5 * ds.x, b.y + (R)0.5 * ds.y, b.z + (R)0.5 * ds.z});
        store3(r.S[(r.parity + k + 1) & 1], i, sn);
    }
    if ((r.flags & kRecord) && w.block == 0 && k > 0)
        finalize_record(r, k - 1, red);
}

// Record from the MEASURE predictor's partials: mode 0 = last step of the
// chunk (slot nsteps - 1), mode 1 = current state (slot 0).
template <typename R>
__global__ __launch_bounds__(kBlockSites) void k_finalize_tail(const ReplicaDev<R>* __restrict__ reps,
                                                               int mode)
{
    __shared__ double red[4][kBlockSites / 64];
    const ReplicaDev<R>& r = reps[blockIdx.x];
    if (!(r.flags & kRecord) || (mode == 0 && r.nsteps <= 0))
        return;
    finalize_record(r, mode == 0 ? r.nsteps - 1 : 0, red);
}

// End of a chunk: advance the step counter and the ping-pong parity.
template <typename R>
__global__ void k_advance(ReplicaDev<R>* __restrict__ reps, int n_rep)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_rep) {
        const int ns = reps[j].nsteps;
        if (ns > 0) {
            reps[j].step += (uint64_t)ns;
            reps[j].parity = (reps[j].parity + ns) & 1;
            if (reps[j].flags & kRecordSeries)
                reps[j].rec_pos += ns;
        }
    }
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
    if (j >= n_rep)
        return;
    const ReplicaDev<R>& r = reps[j];
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

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
template <typename R>
hipError_t launch_predict(const ReplicaDev<R>* reps, const WorkItem* work, const int* n_work,
                          int grid, int k, int remap, bool measure, hipStream_t st)
{
    if (grid <= 0)
        return hipSuccess;
    if (measure)
        hipLaunchKernelGGL((k_predict<R, true>), dim3(grid), dim3(kBlockSites), 0, st, reps, work,
                           n_work, k, remap);
    else
        hipLaunchKernelGGL((k_predict<R, false>), dim3(grid), dim3(kBlockSites), 0, st, reps, work,
                           n_work, k, remap);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_correct(const ReplicaDev<R>* reps, const WorkItem* work, const int* n_work,
                          int grid, int k, int remap, hipStream_t st)
{
    if (grid <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_correct<R>), dim3(grid), dim3(kBlockSites), 0, st, reps, work, n_work, k,
                       remap);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_finalize_tail(const ReplicaDev<R>* reps, int n_rep, int mode, hipStream_t st)
{
    if (n_rep <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_finalize_tail<R>), dim3(n_rep), dim3(kBlockSites), 0, st, reps, mode);
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
                                          int, bool, hipStream_t);                                   \
    template hipError_t launch_correct<R>(const ReplicaDev<R>*, const WorkItem*, const int*, int, int, \
                                          int, hipStream_t);                                         \
    template hipError_t launch_accumulate<R>(const ReplicaDev<R>*, int, hipStream_t);                \
    template hipError_t launch_finalize_tail<R>(const ReplicaDev<R>*, int, int, hipStream_t);             \
    template hipError_t launch_advance<R>(ReplicaDev<R>*, int, hipStream_t);                         \
    template hipError_t launch_noise<R>(uint64_t, uint64_t, int, double*, hipStream_t);

SLLG_INSTANTIATE(float)
SLLG_INSTANTIATE(double)

}  // namespace sllg
