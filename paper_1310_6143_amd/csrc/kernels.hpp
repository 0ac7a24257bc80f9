// Host-side launchers of the HIP kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.hpp"

namespace sllg {

// Predictor of step k of the current chunk over all work items.  With
// measure it only evaluates m and E: of the state after the chunk (k = 0) or
// of the current state (k = 1).
// `grid` workgroups are launched; those whose (remapped) index is at or past
// *n_work (device memory) exit at once, so a captured graph can serve any
// batch up to `grid` blocks.
// variant selects the kernels: 0 uniform materials only, 1 also per-site
// materials and easy axes, 2 also exchange tensors and cubic anisotropy (the
// highest any replica of the batch needs).
template <typename R>
hipError_t launch_predict(const ReplicaDev<R>* reps, const WorkItem* work, const int* n_work,
                          int grid, int k, int remap, bool measure, int variant, hipStream_t st);
// Corrector of step k of the current chunk.
template <typename R>
hipError_t launch_correct(const ReplicaDev<R>* reps, const WorkItem* work, const int* n_work,
                          int grid, int k, int remap, int variant, hipStream_t st);
// Thermal-average block sums of every replica with kAverage.
template <typename R>
hipError_t launch_accumulate(const ReplicaDev<R>* reps, int n_rep, hipStream_t st);
// Completes the record of the measuring predictor's state for every
// recording replica: mode 0 = the chunk's last step (slot nsteps - 1),
// mode 1 = the current state (record slot `slot`).
template <typename R>
hipError_t launch_finish(const ReplicaDev<R>* reps, int n_rep, int mode, int slot, hipStream_t st);
// Step counter and ping-pong parity update at the end of a chunk.
template <typename R>
hipError_t launch_advance(ReplicaDev<R>* reps, int n_rep, hipStream_t st);
// Thermal normals of sites 0..n-1 at one step, as the step kernels draw them.
template <typename R>
hipError_t launch_noise(uint64_t seed, uint64_t step, int n, double* out, hipStream_t st);

// Sites the fixed no-allocation scratch holds (3 doubles each).
constexpr int64_t kNoAllocMaxSites = int64_t(1) << 18;
// Device address and size of the fixed scratch on `device`, looked up once
// per device (with that device current) and kept until the process ends.
hipError_t noalloc_scratch(int device, void** ptr, size_t* bytes);

// Largest torque |S_i x H_i| (deterministic field) of the current state of
// each replica, over the tiles listed in `work` (grid workgroups), into
// out[q] for q < n_rep.  Every tile of a replica with tiles must be listed.
template <typename R>
hipError_t launch_torque(const ReplicaDev<R>* reps, const WorkItem* work, const int* n_work, int grid,
                         int n_rep, int variant, double* out, hipStream_t st);

// Macrocell demagnetising field of the replica at *rep from its current
// state: cell moments, partial dipole sums over `chunks` source ranges
// (dm_part, chunks as allocated for the replica), then the field of every
// cell (dm_field).
template <typename R>
hipError_t launch_demag(const ReplicaDev<R>* rep, int cells, int chunks, hipStream_t st);

// Workgroups of the step kernels that fit on the device at once
// (compute units x resident blocks per unit); 0 if it cannot be queried.
template <typename R>
int resident_blocks(int device, int variant);

// One Monte Carlo sweep of one colour class (count sites listed in
// `sites`) of the replica at *rep, step number `step` for the counters;
// cone = sigma_g, inv_kT = 1/(kB T) (0 at T = 0); accepted trials are added
// to *accepted.  tensor: the replica has exchange tensors (kernel variant
// that applies them).  pids: the stencil pattern of each of the count
// sites, in the same order (required for the stencil forms, else null).
template <typename R>
hipError_t launch_mc(const ReplicaDev<R>* rep, const int32_t* sites, const uint16_t* pids, int count, uint64_t step,
                     double cone, double inv_kT, unsigned long long* accepted, bool tensor, hipStream_t st);

// Fused plane-marching Heun step (fused.hip) of step k over the work items
// (one launch per step; measure: m and E sums of the state after the chunk
// instead, for k_fused_finish).  rec: some replica of the launch takes
// records (false runs the kernel built without the record code; only valid
// when none does, or at k = 0, where no step leaves record sums).  kind:
// FusedKind of every replica of the launch, nb its sites per cell, bt
// threads per workgroup (fused_block_ok); plane_bytes: LDS bytes of one
// plane, the largest over the replicas.
template <typename R>
hipError_t launch_fused(const ReplicaDev<R>* reps, const FusedItem* items, const int* n_items, int grid, int k,
                        int remap, bool measure, bool rec, int kind, int nb, int bt, int plane_bytes, hipStream_t st);
// The end of a fused chunk for every replica: its last two records (when
// recording), the averaging sums of its records, and the advance of the
// step counter, parity and record position.
template <typename R>
hipError_t launch_fused_finish(ReplicaDev<R>* reps, int n_rep, hipStream_t st);
// Monte Carlo records on the fused step's items: after launch_fused with
// measure and k = -1 (the current state, in place), the items' sums of
// every recording replica into record `slot`.
template <typename R>
hipError_t launch_fused_record(ReplicaDev<R>* reps, int n_rep, int slot, hipStream_t st);
// Resident workgroups of the fused kernel (kind, nb, bt) per device with
// plane_bytes LDS planes; 0 if unknown.
template <typename R>
int fused_resident_blocks(int device, int kind, int nb, int bt, int plane_bytes);
// Whether a fused kernel of this kind, block size and precision (bytes per
// real) is built.
bool fused_block_ok(int kind, int bt, size_t real_bytes);
// Dynamic LDS of a fused workgroup with planes of plane_bytes.
size_t fused_lds_bytes(int kind, int plane_bytes, int bt);
// Static LDS of a fused workgroup of bt threads (its FP64 sums, copy table
// and reduction slots).
size_t fused_static_lds(int bt, size_t real_bytes);

// LDS planes of the fused step for a thread region of px x py cells (tile
// plus ring) with nb sites per cell: the region and one more ring.  FP32:
// 16 bytes per site (x, y, z, an unused word), sites basis-major, row after
// row.  FP64: rows of fused_row_slots sites (at least the region's width),
// 32 bytes per site: a row's x, y (16 bytes per site) and then its z (16
// bytes per site, the second word unused).  Planes are filled by
// direct-to-LDS loads of 16 bytes per lane, 64 lanes (1 KiB) per chunk.
constexpr int fused_row_slots(size_t real_bytes, int bt) { return real_bytes == 4 ? 0 : (bt == 256 ? 16 : 32); }
// Chunks of a plane one wave copies at most.
constexpr int fused_chunks_per_wave(size_t real_bytes) { return real_bytes == 4 ? 3 : 6; }
constexpr int fused_plane_bytes(int px, int py, int nb, size_t real_bytes, int bt)
{
    return real_bytes == 4 ? (px + 2) * (py + 2) * nb * 16 : nb * (py + 2) * fused_row_slots(real_bytes, bt) * 32;
}
constexpr int fused_plane_chunks(int px, int py, int nb, size_t real_bytes, int bt)
{
    return (fused_plane_bytes(px, py, nb, real_bytes, bt) + 1023) / 1024;
}
// LDS one workgroup may take on the device.
size_t fused_lds_limit(int device);

hipError_t launch_scatter_records(const double* rec, int count, double* m_dev, double* E_dev,
                                  hipStream_t st);

}  // namespace sllg
