// Host-side builders of the paper's test structures as CSR neighbour lists
// (the appendix on atomistic system generation: a unit cell replicated on a
// grid of cells, optionally cut to a shape, every site's interactions from
// the cell's neighbour template).  Setup only: no device work.
//
// Site numbering and link types follow the cell-by-cell declaration of
// sllg_set_lattice (site i = b + n_basis (x + cells[0] (y + cells[1] z))),
// so a built simple-cubic or bcc block can be declared as a lattice and take
// the fused step.  Rows are sorted by column, then type.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sllg.h"
#include "layout.hpp"
#include "prepare.hpp"

using sllg::kColBits;

namespace {

struct Built {
    std::vector<int64_t> row_ptr{0};
    std::vector<int32_t> col;
    std::vector<uint8_t> type;
    std::vector<double> pos;   // 3 per site, units of the cubic cell edge a
};

// Row of site i: (column, type) pairs sorted by column, then type.
void push_row(Built& out, std::vector<std::pair<int64_t, int>>& row)
{
    std::sort(row.begin(), row.end());
    for (const auto& e : row) {
        out.col.push_back((int32_t)e.first);
        out.type.push_back((uint8_t)e.second);
    }
    out.row_ptr.push_back((int64_t)out.col.size());
    row.clear();
}

// Cell coordinate c + d on an axis of `len` cells: wrapped on a periodic
// axis, -1 past an open end.
int64_t shift(int64_t c, int d, int64_t len, bool periodic)
{
    int64_t u = c + d;
    if (periodic)
        return ((u % len) + len) % len;
    return (u < 0 || u >= len) ? -1 : u;
}

bool check_grid(const int cells[3], const int periodic[3], int n_basis, std::string& why)
{
    if (!cells || !periodic) {
        why = "cells and periodic must not be NULL";
        return false;
    }
    for (int a = 0; a < 3; ++a) {
        if (cells[a] < 1) {
            why = "every axis needs at least one cell";
            return false;
        }
        if (periodic[a] && cells[a] < 3) {
            why = "a periodic axis needs at least 3 cells (links would join a site to itself or twice)";
            return false;
        }
    }
    const double n = (double)cells[0] * cells[1] * cells[2] * n_basis;
    if (n >= (double)(int64_t(1) << kColBits)) {
        why = "at most 2^28 - 1 sites";
        return false;
    }
    return true;
}

// Simple cubic: one site per cell, its 6 nearest neighbours (type 0).
Built build_sc(const int cells[3], const int periodic[3])
{
    Built out;
    const int64_t lx = cells[0], ly = cells[1], lz = cells[2];
    std::vector<std::pair<int64_t, int>> row;
    const int d[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    for (int64_t z = 0; z < lz; ++z)
        for (int64_t y = 0; y < ly; ++y)
            for (int64_t x = 0; x < lx; ++x) {
                for (const auto& o : d) {
                    const int64_t u = shift(x, o[0], lx, periodic[0] != 0), v = shift(y, o[1], ly, periodic[1] != 0),
                                  w = shift(z, o[2], lz, periodic[2] != 0);
                    if (u >= 0 && v >= 0 && w >= 0)
                        row.emplace_back(u + lx * (v + ly * w), 0);
                }
                push_row(out, row);
                out.pos.insert(out.pos.end(), {(double)x, (double)y, (double)z});
            }
    return out;
}

// Body-centred cubic: corner site b = 0 at (0, 0, 0) and body centre b = 1 at
// (1/2, 1/2, 1/2) of each cell.  The 8 first neighbours at a sqrt(3)/2 are
// the other sublattice (type 0): a corner touches the centres of cells
// c + {-1, 0}^3, a centre the corners of cells c + {0, 1}^3.  With second
// neighbours, the 6 sites of the same sublattice one cell along each axis,
// at distance a (type 1).
Built build_bcc(const int cells[3], const int periodic[3], bool second)
{
    Built out;
    const int64_t lx = cells[0], ly = cells[1], lz = cells[2];
    const bool px = periodic[0] != 0, py = periodic[1] != 0, pz = periodic[2] != 0;
    auto site = [&](int64_t x, int64_t y, int64_t z, int b) { return 2 * (x + lx * (y + ly * z)) + b; };
    std::vector<std::pair<int64_t, int>> row;
    for (int64_t z = 0; z < lz; ++z)
        for (int64_t y = 0; y < ly; ++y)
            for (int64_t x = 0; x < lx; ++x)
                for (int b = 0; b < 2; ++b) {
                    const int lo = b == 0 ? -1 : 0;
                    for (int dz = lo; dz <= lo + 1; ++dz)
                        for (int dy = lo; dy <= lo + 1; ++dy)
                            for (int dx = lo; dx <= lo + 1; ++dx) {
                                const int64_t u = shift(x, dx, lx, px), v = shift(y, dy, ly, py), w = shift(z, dz, lz, pz);
                                if (u >= 0 && v >= 0 && w >= 0)
                                    row.emplace_back(site(u, v, w, 1 - b), 0);
                            }
                    if (second) {
                        const int d[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
                        for (const auto& o : d) {
                            const int64_t u = shift(x, o[0], lx, px), v = shift(y, o[1], ly, py),
                                          w = shift(z, o[2], lz, pz);
                            if (u >= 0 && v >= 0 && w >= 0)
                                row.emplace_back(site(u, v, w, b), 1);
                        }
                    }
                    push_row(out, row);
                    const double h = 0.5 * b;
                    out.pos.insert(out.pos.end(), {x + h, y + h, z + h});
                }
    return out;
}

// Sphere cut from an fcc crystal, centred on a lattice site: the points
// (x, y, z) a/2 with x + y + z even whose distance from the centre is at
// most radius_nm + 1e-9 nm, numbered z-major, then y, then x; 12 nearest
// neighbours at a/sqrt(2) in the bulk (type 0), fewer at the surface.
bool build_fcc_sphere(double a_nm, double radius_nm, Built& out, std::string& why)
{
    if (!(a_nm > 0.0) || !(radius_nm >= 0.0) || !std::isfinite(a_nm) || !std::isfinite(radius_nm)) {
        why = "need a_nm > 0 and radius_nm >= 0, both finite";
        return false;
    }
    const double half = a_nm / 2.0, reach = radius_nm + 1e-9;
    const double mh = std::floor(reach / half) + 1.0;
    if (mh > 1000.0) {   // more than 2^28 sites
        why = "at most 2^28 - 1 sites";
        return false;
    }
    const int64_t m = (int64_t)mh, width = 2 * m + 1;
    auto inside = [&](int64_t x, int64_t y, int64_t z) {
        return ((double)x * x + (double)y * y + (double)z * z) * half * half <= reach * reach;
    };
    // sites in order (z, then y, then x ascending) and their grid keys,
    // ascending too: a neighbour is found by binary search
    std::vector<int64_t> key;
    std::vector<int32_t> px, py, pz;
    for (int64_t z = -m; z <= m; ++z)
        for (int64_t y = -m; y <= m; ++y) {
            // |x| <= xr up to rounding; the exact test decides at the edge
            const double r2 = reach * reach / (half * half) - (double)(y * y + z * z);
            if (r2 < -1.0)
                continue;
            const int64_t xr = std::min<int64_t>(m, (int64_t)std::floor(std::sqrt(std::max(r2, 0.0))) + 1);
            for (int64_t x = -xr; x <= xr; ++x) {
                if (((x + y + z) % 2 + 2) % 2 != 0 || !inside(x, y, z))
                    continue;
                if ((int64_t)key.size() >= (int64_t(1) << kColBits) - 1) {
                    why = "at most 2^28 - 1 sites";
                    return false;
                }
                key.push_back(((z + m) * width + (y + m)) * width + (x + m));
                px.push_back((int32_t)x);
                py.push_back((int32_t)y);
                pz.push_back((int32_t)z);
            }
        }
    const int d[12][3] = {{-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}, {1, 1, 0}, {-1, 0, -1}, {-1, 0, 1},
                          {1, 0, -1},  {1, 0, 1},  {0, -1, -1}, {0, -1, 1}, {0, 1, -1}, {0, 1, 1}};
    std::vector<std::pair<int64_t, int>> row;
    for (size_t i = 0; i < key.size(); ++i) {
        for (const auto& o : d) {
            const int64_t x = px[i] + o[0], y = py[i] + o[1], z = pz[i] + o[2];
            if (x < -m || x > m || y < -m || y > m || z < -m || z > m)
                continue;
            const int64_t k = ((z + m) * width + (y + m)) * width + (x + m);
            const auto it = std::lower_bound(key.begin(), key.end(), k);
            if (it != key.end() && *it == k)
                row.emplace_back((int64_t)(it - key.begin()), 0);
        }
        push_row(out, row);
        out.pos.insert(out.pos.end(), {0.5 * px[i], 0.5 * py[i], 0.5 * pz[i]});
    }
    return true;
}

// The two-call protocol shared by the builders: counts only (arrays NULL),
// or a copy into the caller's arrays sized by the counts.
sllg_status deliver(const Built& b, int64_t* n, int64_t* nnz, int64_t* row_ptr, int32_t* col, uint8_t* type,
                    double* pos)
{
    const int64_t nn = (int64_t)b.row_ptr.size() - 1, ne = (int64_t)b.col.size();
    if (!row_ptr && !col && !type && !pos) {
        *n = nn;
        *nnz = ne;
        return SLLG_OK;
    }
    if (!row_ptr || !col) {
        sllg::set_create_error("row_ptr and col are both needed (type and pos may be NULL)");
        return SLLG_E_ARG;
    }
    if (*n != nn || *nnz != ne) {
        sllg::set_create_error("*n and *nnz must hold the counts of the first call (" + std::to_string(nn) + ", " +
                               std::to_string(ne) + ")");
        return SLLG_E_ARG;
    }
    std::memcpy(row_ptr, b.row_ptr.data(), (size_t)(nn + 1) * sizeof(int64_t));
    if (ne)
        std::memcpy(col, b.col.data(), (size_t)ne * sizeof(int32_t));
    if (type && ne)
        std::memcpy(type, b.type.data(), (size_t)ne);
    if (pos && nn)
        std::memcpy(pos, b.pos.data(), (size_t)(3 * nn) * sizeof(double));
    return SLLG_OK;
}

template <typename F>
sllg_status guarded(int64_t* n, int64_t* nnz, F&& fn)
{
    if (!n || !nnz) {
        sllg::set_create_error("n and nnz must not be NULL");
        return SLLG_E_ARG;
    }
    try {
        return fn();
    } catch (const std::bad_alloc&) {
        sllg::set_create_error("out of host memory");
        return SLLG_E_NOMEM;
    } catch (...) {
        sllg::set_create_error("builder failed");
        return SLLG_E_ARG;
    }
}

}  // namespace

extern "C" {

sllg_status sllg_build_sc(const int cells[3], const int periodic[3], int64_t* n, int64_t* nnz, int64_t* row_ptr,
                          int32_t* col, uint8_t* type, double* pos)
{
    return guarded(n, nnz, [&] {
        std::string why;
        if (!check_grid(cells, periodic, 1, why)) {
            sllg::set_create_error(why);
            return SLLG_E_ARG;
        }
        return deliver(build_sc(cells, periodic), n, nnz, row_ptr, col, type, pos);
    });
}

sllg_status sllg_build_bcc(const int cells[3], const int periodic[3], int second_neighbours, int64_t* n,
                           int64_t* nnz, int64_t* row_ptr, int32_t* col, uint8_t* type, double* pos)
{
    return guarded(n, nnz, [&] {
        std::string why;
        if (!check_grid(cells, periodic, 2, why)) {
            sllg::set_create_error(why);
            return SLLG_E_ARG;
        }
        return deliver(build_bcc(cells, periodic, second_neighbours != 0), n, nnz, row_ptr, col, type, pos);
    });
}

sllg_status sllg_build_fcc_sphere(double a_nm, double radius_nm, int64_t* n, int64_t* nnz, int64_t* row_ptr,
                                  int32_t* col, uint8_t* type, double* pos)
{
    return guarded(n, nnz, [&] {
        Built b;
        std::string why;
        if (!build_fcc_sphere(a_nm, radius_nm, b, why)) {
            sllg::set_create_error(why);
            return SLLG_E_ARG;
        }
        return deliver(b, n, nnz, row_ptr, col, type, pos);
    });
}

}  // extern "C"
