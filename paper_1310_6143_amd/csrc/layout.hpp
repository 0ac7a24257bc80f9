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
// Wide stencil form (kWide): patterns and entries (all patterns padded to
// the longest) it takes at most.
constexpr int kWideMaxPatterns = 65535;
constexpr int kWideMaxEntries = 1 << 22;
// A wide-form entry packs (column - row) << 5 | type; type kMaxTypes (J = 0)
// pads each pattern's near and far parts to whole batches of kWideBatch.
constexpr int kWideBatch = 8;
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
    kFused = 4096,          // the lattice runs the fused plane-marching step (f_* fields)
    kWide = 8192,           // neighbours in the wide stencil form (w_pid / w_tab in global memory)
};

// Rows longer than this take the batched gathers of the general variant.
constexpr int kLongRow = 32;

// Flags that need the general (per-site) kernel variant.
constexpr int32_t kGeneralFlags = kPerSiteMaterial | kPerSiteAxis | kTensor | kCubic | kDemag | kLongRows;
// Flags that need variant 2 (exchange tensors, cubic anisotropy,
// demagnetising field, long rows).
constexpr int32_t kVariant2Flags = kTensor | kCubic | kDemag | kLongRows;

// Fused plane-marching step (one launch per Heun step).  A lattice of nb
// sites per cell on an nx x ny x nz grid of cells, site i = b + nb (x + nx
// (y + ny z)), periodic in x and y, periodic or open in z, whose links join
// cells at most one cell apart on every axis.  A work item is a tile of
// columns marched through a range of planes; its workgroup holds one plane
// of S and one of S' in LDS, one thread per column of the tile and a ring
// of one cell around it (the predictor is recomputed on the ring so that
// the corrector of the tile needs no other workgroup).
constexpr int kFusedMaxPatterns = 64;     // distinct (plane class, basis site) link patterns
constexpr int kFusedMaxEntries = 1024;    // entries of all patterns together
constexpr int kFusedMaxBasis = 2;         // sites per cell the fused kernels are built for
constexpr int kFusedMinEdge = 8;          // smallest thread region per axis (cells)

// Lattice kinds the fused kernel is compiled for, so that a site's links
// are compile-time constants (LDS offsets become instruction immediates):
// simple cubic with 6 nearest neighbours; bcc with its 8 nearest neighbours
// (type slot 0); bcc with the 6 second neighbours as well (slot 1).  A link
// is (dz, dy, dx, bp): the neighbour is basis site bp of the cell offset by
// (dx, dy, dz).  Kind 0 is any other lattice the fused step takes, its
// links read from a table at run time.
enum FusedKind : int32_t { kKindGeneric = 0, kKindSc6 = 1, kKindBcc8 = 2, kKindBcc14 = 3 };

__host__ __device__ constexpr int kind_basis(int kind)
{
    return kind == kKindSc6 ? 1 : (kind == kKindBcc8 || kind == kKindBcc14) ? 2 : 0;
}

// Whether basis site b of `kind` has the link (dz, dy, dx, bp); its type
// slot goes to *slot.  Enumerating dz, dy, dx, bp in increasing order
// lists the links in the canonical order the fused step sums them in.
__host__ __device__ constexpr bool kind_link(int kind, int b, int dz, int dy, int dx, int bp, int* slot)
{
    const int manhattan = (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz);
    if (kind == kKindSc6) {
        *slot = 0;
        return bp == 0 && manhattan == 1;
    }
    if (kind == kKindBcc8 || kind == kKindBcc14) {
        // site 0 at cell c touches the body centres (site 1) of cells
        // c + {-1, 0}^3; site 1 touches the corners (site 0) of c + {0, 1}^3
        const int lo = b == 0 ? -1 : 0;
        if (bp != b && dx >= lo && dx <= lo + 1 && dy >= lo && dy <= lo + 1 && dz >= lo && dz <= lo + 1) {
            *slot = 0;
            return true;
        }
        if (kind == kKindBcc14 && bp == b && manhattan == 1) {
            *slot = 1;
            return true;
        }
    }
    return false;
}

// A pattern entry: byte offset of the neighbour's LDS slot from the site's
// own (for the replica's region width) and J / mu_ref.
struct FusedEntry {
    int32_t off;
    float J;
};
struct FusedEntryD {
    int32_t off;
    int32_t pad;
    double J;
};

struct FusedItem {
    int32_t replica;
    int32_t x0, y0;      // first cell of the tile (interior) on x and y
    int32_t z0, z1;      // planes the item integrates: [z0, z1)
    int32_t idx;         // item number within its replica (slot of its partials)
};

template <typename R>
struct ReplicaDev {
    R* S[2];                        // ping-pong spin buffers [3n]
    R* Sp;                          // predicted spins S' [3n]
    int32_t* fault;                 // set to 1 by a kernel that produced a non-finite spin (cleared with new spins)
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
    int32_t w_len;                  // entries per pattern in the wide form (kWide)
    const uint16_t* w_pid;          // [n] pattern of each site (kWide)
    const int32_t* w_tab;           // [w_len][n_patterns] packed offset << 5 | type, transposed (kWide)
    const uint16_t* w_near;         // [n_patterns] near entries of each pattern, padded to kWideBatch (kWide)
    // fused plane-marching step (kFused)
    const void* f_ent;              // FusedEntry (FP32) / FusedEntryD (FP64) of every pattern
    const int32_t* f_pat;           // [patterns][4]: first entry, entries with dz = -1, 0, +1
    const uint8_t* f_plane;         // [nz][nb] pattern of each (plane, basis site); null: pattern = basis site
    double* f_partials;             // [2][f_items][4] m and E sums per item, by step parity
    int32_t f_nb;                   // sites per cell
    int32_t f_nx, f_ny, f_nz;       // cells per axis
    int32_t f_zper;                 // 1: periodic in z
    int32_t f_px, f_py;             // thread region per axis: tile + 2 cells
    int32_t f_items;                // work items of the replica
    int32_t f_npat;                 // patterns
    int32_t f_nent;                 // pattern entries
    int32_t f_kind;                 // FusedKind of the lattice
    int32_t f_pad;
    R f_kj[2];                      // J / mu_ref of the kind's type slots
};

struct WorkItem {
    int32_t replica;
    int32_t block;                  // tile index within the replica
};

}  // namespace sllg
