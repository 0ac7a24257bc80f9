// Host-side preparation of a spin system for the device: validation of the
// caller's CSR neighbour list and material arrays, conversion of the CSR to
// the SELL-64 layout the step kernels read, and the material table.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sllg.h"
#include "layout.hpp"

namespace sllg {

// Internal failure carrying an ABI status; caught at the C boundary.
struct Failure {
    sllg_status code;
    std::string msg;
};

[[noreturn]] void fail(sllg_status code, const std::string& msg);

// Boltzmann constant (J/K), Table 1 of the paper.
constexpr double kBoltzmann = 1.3807e-23;
// Bohr magneton (J/T), Table 1 of the paper.
constexpr double kBohrMagneton = 9.2740e-24;

// Macrocell decomposition for the demagnetising field: cubic cells of edge
// cell_size on a grid that starts a thousandth of a cell below the smallest
// atom coordinate on each axis (atomic planes on a cell boundary go to the
// upper cell); cells are numbered in the order of (x, y, z) cell index.
struct HostDemag {
    bool on = false;
    double cell_size = 0.0, atom_volume = 0.0;
    int64_t every = 1;
    int64_t cells = 0;
    std::vector<double> pos;           // [3n] atom positions relative to the grid corner (m)
    std::vector<int32_t> cell_of;      // [n]
    std::vector<int32_t> start;        // [cells + 1]
    std::vector<int32_t> atoms;        // [n] sites sorted by cell, ascending within a cell
};

// Source chunks of the demagnetising-field update: enough workgroups
// (blocks of 256 cells x chunks, about 2048) to fill the chip, at most 32.
inline int demag_chunks(int64_t cells)
{
    const int64_t blocks = (cells + 255) / 256;
    const int64_t c = (2048 + blocks - 1) / (blocks > 0 ? blocks : 1);
    return (int)(c < 1 ? 1 : (c > 32 ? 32 : c));
}

// Validates and builds the decomposition (pos: 3n metres).
HostDemag build_demag(int64_t n, const double* pos, double cell_size, double atom_volume, int64_t every);

// A lattice declared cell by cell (sllg_set_lattice): site
// i = b + nb (x + nx (y + ny z)); every link joins cells at most one cell
// apart on each axis (across the boundary of a periodic axis).  The fused
// step keeps one link pattern per (plane, basis site).
struct FusedLink {
    int8_t dz, dy, dx;      // cell offset of the neighbour
    uint8_t bp;             // its basis site
    uint8_t type;           // interaction type
    bool operator<(const FusedLink& o) const
    {
        if (dz != o.dz) return dz < o.dz;
        if (dy != o.dy) return dy < o.dy;
        if (dx != o.dx) return dx < o.dx;
        if (bp != o.bp) return bp < o.bp;
        return type < o.type;
    }
    bool operator==(const FusedLink& o) const
    {
        return dz == o.dz && dy == o.dy && dx == o.dx && bp == o.bp && type == o.type;
    }
};

struct HostLattice {
    bool on = false;
    int nb = 0, nx = 0, ny = 0, nz = 0;
    bool per[3] = {false, false, false};
    bool fusable = false;                       // the fused step can run on this structure
    std::string why;                            // why not, when it cannot
    std::vector<std::vector<FusedLink>> pats;   // link patterns, each sorted (dz first)
    std::vector<uint8_t> pat_b;                 // basis site of each pattern
    std::vector<uint8_t> plane_pat;             // [nz * nb] pattern of each (plane, basis site);
                                                // empty when the pattern is the basis site itself
    int kind = 0;                               // FusedKind whose links every site has (kKindGeneric: none)
    int slot_type[2] = {0, 0};                  // interaction type of each of the kind's slots
};

// Sets the error text of the calls without a handle (sllg_last_error(NULL)).
void set_create_error(const std::string& msg);

// Whether the fused step is built for lattice L of n sites in a precision
// (bytes per real): FP32 any fusable lattice, FP64 the compiled kinds; the
// spins must be addressable with 31-bit byte offsets.
inline bool fused_precision_ok(const HostLattice& L, int64_t n, size_t real_bytes)
{
    return L.on && L.fusable && (real_bytes == 4 || L.kind != kKindGeneric) && n * 3 * (int64_t)real_bytes + 16 <= 0x7FFFFFFF;
}

// Neighbour structure in stencil or SELL-64 form.  Every row lists its
// near links (|col - row| <= halo_cap) first and the far ones after, each
// part in the caller's order; the step kernels sum the two parts separately
// (near ones from the LDS window), so both forms add the same terms in the
// same order.
struct HostStructure {
    int64_t n = 0;
    int64_t nnz = 0;
    int n_types = 0;
    int halo = 0;                      // window halo: max near |col - row|, rounded up to 4
    int tile_request = 0;              // sites per tile: 0 from n (tile_for), -1 the largest, else this
    std::vector<double> J;             // joules per link, per type
    // exchange tensors (set_exchange_tensors): 9 per type, row-major, joules
    bool tensor = false;
    std::vector<double> Jt;
    // reverse[t] bit u: some link of type t has its reverse link of type u
    // (recorded by the symmetry check; rev_known = false without it)
    bool rev_known = false;
    uint16_t reverse[kMaxTypes] = {};
    std::vector<uint32_t> nb;          // packed entries, 64 rows per slice, column-major
    std::vector<int64_t> slice_off;    // [n_slices + 1]
    std::vector<uint32_t> deg;         // [n] near << 16 | degree
    bool long_rows = false;            // SELL rows longer than kLongRow links
    // stencil form, filled when every row matches one of few patterns
    bool stencil = false;
    std::vector<uint8_t> pat_id;       // [n]
    std::vector<int32_t> pat_tab;      // packed (col - row) << 4 | type
    std::vector<uint16_t> pat_start;   // [n_patterns + 1]
    std::vector<uint16_t> pat_far;     // [n_patterns] first far entry of each pattern
    bool no_far = false;               // no pattern has a far link (no padding then)
    // wide stencil form, filled when the patterns exceed the LDS tables
    // (kMaxPatterns, kMaxPatternEntries) but not kWideMaxPatterns /
    // kWideMaxEntries: the table stays in global memory
    bool wide = false;
    int w_len = 0;                     // entries of the longest pattern (a multiple of kWideBatch)
    std::vector<uint16_t> w_pid;       // [n] pattern of each site
    std::vector<int32_t> w_tab;        // [w_len][patterns] packed (col - row) << 5 | type: the near links,
                                       // padded to kWideBatch, then the far ones, padded (type kMaxTypes)
    std::vector<uint16_t> w_near;      // [patterns] near entries of each pattern with their padding
    // macrocell demagnetising field (set_demag)
    HostDemag demag;
    // Monte Carlo colour classes (build_colours): sites sorted by colour
    std::vector<int32_t> colour_sites;
    std::vector<int64_t> colour_start;   // [n_colours + 1]
    // lattice declaration and fused-step patterns (set_lattice)
    HostLattice lat;
};

// Declares the structure's sites as a lattice of nb sites per cell on
// cells[0] x cells[1] x cells[2] cells (periodic[a] != 0: periodic axis) and
// derives the fused step's link patterns.  Throws Failure(SLLG_E_ARG) when
// the counts do not match or a link joins cells more than one cell apart;
// otherwise sets s.lat (fusable false, with the reason, when the fused step
// cannot take the structure: open x or y, patterns that change within a
// plane, more than 2 sites per cell, too many patterns).
void set_lattice(HostStructure& s, int nb, const int cells[3], const int periodic[3]);

// Sites per tile of this structure at a precision (see tile_request).
int tile_of(const HostStructure& s, size_t real_bytes);

// Validates and converts.  Throws Failure(SLLG_E_ARG) on malformed input.
// allow_stencil = false keeps the SELL form even when patterns would fit
// (LDS stencil or wide stencil).
// halo_cap (a multiple of 4) bounds the offsets read from the LDS window.
HostStructure build_structure(int64_t n, const int64_t* row_ptr, const int32_t* col,
                              const uint8_t* ntype, const double* J, int n_types,
                              bool check_symmetry, int halo_cap, bool allow_stencil = true);

// Exchange tensors for the types of s (n_types must match).  With the
// symmetry check's record, every link of type t whose reverse has type u
// needs Jt[u] = Jt[t]^T, so the energy -S_i^T J_ij S_j is the same read
// from either end.  Jt = NULL returns to the scalar table.
void set_exchange_tensors(HostStructure& s, const double* Jt, int n_types);

// Greedy colouring of the neighbour graph for Monte Carlo: the sites are
// visited in ascending order, or (lattice_order, on a declared lattice)
// grouped by basis site and by the parity of the cell's x + y + z, each
// taking the smallest colour no earlier-visited neighbour has (so no link
// joins two sites of one colour); fills colour_sites / colour_start.
void build_colours(HostStructure& s, bool lattice_order);

// Materials: distinct (mu_s, k_u, k_c) triples, per-site ids when there is
// more than one, per-site easy axes when they differ.
struct HostMaterials {
    int64_t n = 0;
    std::vector<double> mat_mu;        // J/T per material
    std::vector<double> mat_ku;        // J per material
    std::vector<double> mat_kc;        // J per material (cubic anisotropy)
    bool cubic = false;                // some k_c != 0
    double axis[3] = {0, 0, 1};        // uniform easy axis (when !per_site_axis)
    std::vector<uint8_t> matid;        // [n] when per_site_material
    std::vector<double> axis_site;     // [3n] when per_site_axis
    bool per_site_material = false;
    bool per_site_axis = false;
    double mu_ref = 0.0;               // reference moment for the field units
    double mu_total = 0.0;             // sum over sites of mu_s
};

// Per demagnetising macrocell: magnetic centre of mass sum mu x / sum mu (3
// per cell, relative to the grid corner) and the self-field factor
// mu0 / (3 V), V = atoms * atom_volume.
void demag_cells(const HostDemag& dm, const HostMaterials& m, std::vector<double>& centre,
                 std::vector<double>& self);

// k_c: cubic anisotropy, n values when kc_per_site, else one (NULL: none).
HostMaterials build_materials(int64_t n, const double* mu_s, const double* k_u,
                              const double* easy_axis, int per_site, const double* k_c = nullptr,
                              int kc_per_site = 0);

// Validate spins (3n doubles; throws on zero or non-finite length) and
// normalise them, or with normalise = false copy them unchanged (a restored
// checkpoint continues bit for bit).
std::vector<double> normalised_spins(int64_t n, const double* S, bool normalise = true);

// Integration parameters of one replica.
struct Dynamics {
    double alpha = -1.0, gamma = -1.0, dt = -1.0;
    double temperature = 0.0;
    double H[3] = {0.0, 0.0, 0.0};
    uint64_t seed = 0;
    uint64_t step = 0;
};

void check_dynamics(const Dynamics& d);

// Device material table for the current dynamics (thermal width depends on
// lambda, T, gamma and dt).
template <typename R>
std::vector<MaterialDev<R>> material_table(const HostMaterials& m, const Dynamics& d);

// Fill the parameter part of a replica record (J table, gamma dt, field, ...).
template <typename R>
void fill_parameters(ReplicaDev<R>& rec, const HostStructure& s, const HostMaterials& m,
                     const Dynamics& d);

// Thermal averages from per-block sums acc[b][5] = sums of (|m|, m_x, m_y,
// m_z, E) over block_len samples each: out = { <|m|>, se, <m_x>, <m_y>,
// <m_z>, <E>, se(E), n_blocks }, se = std of the block means / sqrt(n_blocks).
void averages_from_block_sums(const double* acc, int n_blocks, int64_t block_len, double out[8]);

}  // namespace sllg
