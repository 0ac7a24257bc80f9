// Device-side data layout of libsllg, shared by the kernels and the host
// runtime.  Holds plain structs only.
//
// One "replica" is one independent spin system.  A single system created
// through sllg_create is a batch of one replica; the server batches many.
// Every replica owns its device buffers; the kernels find them through a
// table of ReplicaDev records, and a table of work items maps each tile of
// consecutive sites of a replica to the workgroup that sweeps it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sllg {

// Step kernels: workgroups of kBlockThreads lanes sweep tiles of
// consecutive sites (tile_for(): a few sites per lane).
// A workgroup stages its tile's spins plus a halo of up to kHaloCap sites
// on either side in LDS; neighbours within the halo are read from there,
// the rest from global memory.
#ifndef SLLG_TILE_SITES_F32
#define SLLG_TILE_SITES_F32 2048
#endif
#ifndef SLLG_TILE_SITES_F64
#define SLLG_TILE_SITES_F64 1024
#endif
#ifndef SLLG_HALO_CAP
#define SLLG_HALO_CAP 384
#endif
#ifndef SLLG_BLOCK_THREADS
#define SLLG_BLOCK_THREADS 512
#endif
constexpr int kBlockThreads = SLLG_BLOCK_THREADS;
// Largest tile (the LDS arrays are sized for it).
template <typename R>
constexpr int tile_sites()
{
    return sizeof(R) == 4 ? SLLG_TILE_SITES_F32 : SLLG_TILE_SITES_F64;
}
// Tiles a replica should have at least, so that small systems still spread
// over the whole chip.
#ifndef SLLG_MIN_TILES
#define SLLG_MIN_TILES 2048
#endif
constexpr int64_t kMinTiles = SLLG_MIN_TILES;
// Tile size of an n-site replica: the largest power-of-two fraction of the
// largest tile (down to one site per lane) that still gives kMinTiles
// tiles.  A function of n and the precision only, so a replica is tiled the
// same way alone and in any batch.
__host__ __device__ inline int tile_for(int64_t n, size_t real_bytes)
{
    int t = real_bytes == 4 ? SLLG_TILE_SITES_F32 : SLLG_TILE_SITES_F64;
    while (t > kBlockThreads && (n + t - 1) / t < kMinTiles)
        t /= 2;
    return t;
}
constexpr int kHaloCap = SLLG_HALO_CAP;
static_assert(SLLG_TILE_SITES_F32 % kBlockThreads == 0 && SLLG_TILE_SITES_F64 % kBlockThreads == 0 &&
                  (SLLG_TILE_SITES_F32 / kBlockThreads & (SLLG_TILE_SITES_F32 / kBlockThreads - 1)) == 0 &&
                  (SLLG_TILE_SITES_F64 / kBlockThreads & (SLLG_TILE_SITES_F64 / kBlockThreads - 1)) == 0,
              "a tile is a whole number of sites per lane");
static_assert(SLLG_HALO_CAP % 4 == 0, "the halo keeps 16-byte alignment of the staged window");
static_assert(SLLG_BLOCK_THREADS % 64 == 0 && SLLG_BLOCK_THREADS >= 256, "whole wavefronts; a group sum takes one lane per tile");
// Spin buffers are padded to a multiple of 16 bytes so that a tile's
// window is staged with whole 16-byte loads.
__host__ __device__ inline size_t spin_buffer_bytes(int64_t n, size_t real_bytes)
{
    return (3 * (size_t)n * real_bytes + 15) & ~size_t(15);
}
constexpr int kGroupTiles = 256;      // tile partials summed together at the second level
constexpr int kSlice = 64;            // rows per SELL slice = one wavefront
constexpr int kMaxTypes = 16;         // interaction types per replica
constexpr uint32_t kColBits = 28;     // packed neighbour: type << 28 | column
constexpr uint32_t kColMask = (1u << kColBits) - 1u;
constexpr int kMaxDegree = 4095;       // neighbours per site (long-range exchange)
// Stencil format: rows whose (column - row, type) lists coincide share one
// pattern; a site stores only its pattern id (uint8).  Pattern entries pack
// (column - row) << 4 | type in an int32 (offsets within +-2^27).
constexpr int kMaxPatterns = 256;
// Far links of a stencil row the step kernels keep in flight in registers;
// the host pads every pattern's far part to at least this many entries
// (offset 0, J = 0) unless no pattern has any far link.
constexpr int kFarRegs = 6;
#ifndef SLLG_MAX_PATTERN_ENTRIES
#define SLLG_MAX_PATTERN_ENTRIES 1024
#endif
constexpr int kMaxPatternEntries = SLLG_MAX_PATTERN_ENTRIES;   // all patterns' entries, staged in LDS

// Per-material constants, pre-scaled to field units (tesla).
template <typename R>
struct MaterialDev {
    R mu_rel;       // mu_ref / mu_s: exchange field = mu_rel * sum_k jt[type] S_j
    R mu_frac;      // mu_s / mu_ref: weight of the site in m and E
    R ani;          // 2 k_u / mu_s  (anisotropy field factor)
    R ku_mu;        // k_u / mu_s    (anisotropy energy per unit moment)
    R sigma;        // thermal-field width sqrt(2 lambda kB T / (gamma mu_s dt))
    R axis[3];      // easy axis when it is uniform over the material
    R cub;          // -2 k_c / mu_s (cubic anisotropy field factor, kCubic)
    R kc_mu;        // k_c / mu_s    (cubic anisotropy energy per unit moment)
    double mu_s;    // J/T, for the energy and magnetisation sums
};

enum ReplicaFlags : int32_t {
    kPerSiteMaterial = 1,   // matid[] selects the material of each site
    kPerSiteAxis = 2,       // axis[] holds one easy axis per site
    kRecord = 4,            // compute m and E after every step
    kRecordSeries = 8,      // records[] holds the whole run: rec_pos advances per chunk
    kAverage = 16,          // add the records to the thermal-average block sums acc[]
    kStencil = 32,          // neighbours in stencil form (pat_id / pat_tab) instead of SELL
    kNoFar = 64,            // stencil form without far links (every neighbour in the LDS window)
    kDirect = 128,          // no LDS window: every neighbour and the own spin read from global memory
    kTensor = 256,          // exchange tensors jm[type] instead of the scalars jt[type]
    kCubic = 512,           // cubic anisotropy (material fields cub, kc_mu)
    kDemag = 1024,          // macrocell demagnetising field dm_field[dm_cell[i]] added to every site
    kLongRows = 2048,       // SELL rows longer than kLongRow links: batched gathers (general variant)
};

// Rows longer than this take the batched gathers of the general variant.
constexpr int kLongRow = 32;

// Flags that need the general (per-site) kernel variant.
constexpr int32_t kGeneralFlags = kPerSiteMaterial | kPerSiteAxis | kTensor | kCubic | kDemag | kLongRows;
// Flags that need variant 2 (exchange tensors, cubic anisotropy,
// demagnetising field, long rows).
constexpr int32_t kVariant2Flags = kTensor | kCubic | kDemag | kLongRows;

template <typename R>
struct ReplicaDev {
    R* S[2];                        // ping-pong spin buffers [3n]
    R* Sp;                          // predicted spins S' [3n]
    const uint32_t* nb;             // SELL-64 neighbour entries
    const int64_t* slice_off;       // [n_slices + 1] first entry of each slice
    const uint32_t* deg;            // [n] near << 16 | neighbours, per site (SELL)
    const uint8_t* pat_id;          // [n padded to 16] stencil pattern of each site (kStencil)
    const int32_t* pat_tab;         // [pat_entries] packed offset << 4 | type
    const uint16_t* pat_start;      // [n_patterns + 1] first entry of each pattern
    const uint16_t* pat_far;        // [n_patterns] first entry beyond the halo, per pattern
    const uint8_t* matid;           // [n] or null
    const R* axis;                  // [3n] or null
    const MaterialDev<R>* mat;      // materials
    double* partials;               // [blocks][4]: sum mu S (3), energy of each tile
    double* group_partials;         // [groups][4]: sums over kGroupTiles consecutive tiles
    double* records;                // [cap][4] per-step m (3) and E
    double* acc;                    // [avg_blocks][5] sums of |m|, m (3), E per averaging block
    R jt[kMaxTypes];                // J / mu_ref per type (tesla)
    R jm[kMaxTypes][9];             // exchange tensor / mu_ref per type, row-major (kTensor)
    // macrocell demagnetising field (kDemag)
    const int32_t* dm_cell;         // [n] macrocell of each site
    const int32_t* dm_start;        // [cells + 1] first entry of each cell in dm_atoms
    const int32_t* dm_atoms;        // [n] sites sorted by cell
    const R* dm_pos;                // [3 cells] magnetic centres of mass (m, from the grid corner)
    const R* dm_self;               // [cells] mu0 / (3 V) of each cell: self field per unit moment
    R* dm_m;                        // [3 cells] cell moments (J/T)
    R* dm_field;                    // [3 cells] field of the last update (T)
    R* dm_part;                     // [chunks][3 cells] partial dipole sums over one chunk of cells q
    int32_t dm_cells;
    int32_t dm_chunks;              // chunks the sources q are split into (parallelism of the update)
    R gdt;                          // gamma / (1 + lambda^2) * dt
    R alpha;                        // lambda
    R H[3];                         // applied field (T)
    double inv_mu_total;            // 1 / sum_i mu_s,i
    double mu_ref;                  // unit of the per-site m and E terms (J/T)
    uint64_t seed;                  // Philox key
    uint64_t step;                  // number of the next step (advanced on the device)
    int64_t rec_pos;                // record slot of the chunk's first step
    int64_t avg_first;              // first averaged step number (its post-step state)
    int64_t avg_block_len;          // samples per averaging block
    int32_t avg_blocks;             // number of averaging blocks
    int32_t halo;                   // window halo in sites (multiple of 4, <= kHaloCap)
    int32_t n;                      // sites
    int32_t blocks;                 // tiles: ceil(n / tile)
    int32_t parity;                 // S[parity] holds the current state (advanced on the device)
    int32_t nsteps;                 // steps this replica takes in the current chunk
    int32_t flags;                  // ReplicaFlags
    int32_t n_patterns;             // stencil patterns (kStencil)
    int32_t tile;                   // sites per tile: tile_for(n, sizeof(R))
    int32_t pad1;
};

struct WorkItem {
    int32_t replica;
    int32_t block;                  // tile index within the replica
};

}  // namespace sllg
