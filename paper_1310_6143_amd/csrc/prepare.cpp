// Host-side validation and layout conversion (see prepare.hpp).
#include "prepare.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <thread>
#include <unordered_map>
#include <tuple>
#include <utility>

namespace sllg {

void fail(sllg_status code, const std::string& msg) { throw Failure{code, msg}; }

int tile_of(const HostStructure& s, size_t real_bytes)
{
    const int largest = real_bytes == 4 ? tile_sites<float>() : tile_sites<double>();
    if (s.tile_request < 0)
        return largest;
    if (s.tile_request == 0)
        return tile_for(s.n, real_bytes);
    return std::min(s.tile_request, largest);
}

HostStructure build_structure(int64_t n, const int64_t* row_ptr, const int32_t* col,
                              const uint8_t* ntype, const double* J, int n_types,
                              bool check_symmetry, int halo_cap, bool allow_stencil)
{
    if (n <= 0)
        fail(SLLG_E_ARG, "system has no spins");
    if (!row_ptr || !J)
        fail(SLLG_E_ARG, "row_ptr and J must not be NULL");
    if (n_types < 1 || n_types > kMaxTypes)
        fail(SLLG_E_ARG, "n_types must be in 1..16");
    for (int t = 0; t < n_types; ++t)
        if (!std::isfinite(J[t]))
            fail(SLLG_E_ARG, "J table holds a non-finite value");
    if (row_ptr[0] != 0)
        fail(SLLG_E_ARG, "row_ptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i) {
        const int64_t d = row_ptr[i + 1] - row_ptr[i];
        if (d < 0)
            fail(SLLG_E_ARG, "row_ptr is decreasing at row " + std::to_string(i));
        if (d > kMaxDegree)
            fail(SLLG_E_ARG, "row " + std::to_string(i) + " has more than " + std::to_string(kMaxDegree) +
                                 " neighbours");
    }
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && !col)
        fail(SLLG_E_ARG, "col must not be NULL");
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int64_t j = col[k];
            if (j < 0 || j >= n)
                fail(SLLG_E_ARG, "column out of range in row " + std::to_string(i));
            if (j == i)
                fail(SLLG_E_ARG, "self link in row " + std::to_string(i));
            if (ntype && ntype[k] >= n_types)
                fail(SLLG_E_ARG, "interaction type out of range in row " + std::to_string(i));
        }
    }
    HostStructure s;
    if (check_symmetry) {
        // every link i -> j of type t needs a reverse link j -> i of a type u
        // with the same coupling (u = t, or a type with an equal J, which
        // exchange tensors may tell apart: the pairs (t, u) are recorded)
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                const int64_t j = col[k];
                const int t = ntype ? ntype[k] : 0;
                int u = -1;
                for (int64_t q = row_ptr[j]; q < row_ptr[j + 1] && u != t; ++q) {
                    const int tq = ntype ? ntype[q] : 0;
                    if (col[q] == i && (u < 0 || tq == t) && J[tq] == J[t])
                        u = tq;
                }
                if (u < 0)
                    fail(SLLG_E_ARG, "link " + std::to_string(i) + "->" + std::to_string(j) +
                                         " has no reverse link with the same J");
                s.reverse[t] |= (uint16_t)(1u << u);
            }
        }
        s.rev_known = true;
    }
    s.n = n;
    s.nnz = nnz;
    s.n_types = n_types;
    s.J.assign(J, J + n_types);
    if (halo_cap < 0 || halo_cap % 4 != 0)
        fail(SLLG_E_ARG, "halo cap must be a non-negative multiple of 4");

    // Row order of the device forms: near links first, then far ones.
    auto near = [&](int64_t i, int64_t q) {
        const int64_t off = (int64_t)col[q] - i;
        return off >= -halo_cap && off <= halo_cap;
    };
    std::vector<int64_t> order((size_t)nnz);   // CSR positions, rows reordered
    std::vector<uint16_t> n_near((size_t)n);
    int64_t max_near = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t w = row_ptr[i];
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
            if (near(i, q)) {
                order[(size_t)w++] = q;
                max_near = std::max<int64_t>(max_near, std::llabs((int64_t)col[q] - i));
            }
        n_near[(size_t)i] = (uint16_t)(w - row_ptr[i]);
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
            if (!near(i, q))
                order[(size_t)w++] = q;
    }
    s.halo = (int)((max_near + 3) & ~int64_t(3));

    // Stencil form: the interaction list of a row, written relative to the
    // row, repeats across a crystal (the paper builds it from the unit
    // cell's neighbour template), so few patterns cover every row.  Up to
    // kMaxPatterns patterns of kMaxPatternEntries entries in all are staged
    // in LDS; more (periodic images of long-range rows: one pattern per
    // combination of boundary distances) take the wide form, whose table
    // stays in global memory (read through the L2), transposed so that the
    // lanes of a wavefront read entry k of their patterns side by side.
    {
        std::unordered_map<std::string, int> ids;
        std::vector<uint16_t> pid((size_t)n);
        std::vector<std::string> keys;   // per pattern: near count, then the packed entries
        std::string key;
        bool ok = allow_stencil && n * 24 <= 0x7FFFF000;
        // Far parts of the LDS form are padded to kFarRegs entries (offset
        // 0: never a real link, self links are rejected above) unless no
        // row has far links.
        bool any_far = false;
        for (int64_t i = 0; i < n && !any_far; ++i)
            any_far = n_near[(size_t)i] < row_ptr[i + 1] - row_ptr[i];
        const size_t far_min = any_far ? (size_t)kFarRegs : 0;
        size_t lds_entries = 0, longest = 0;
        for (int64_t i = 0; i < n && ok; ++i) {
            key.clear();
            key.append(reinterpret_cast<const char*>(&n_near[(size_t)i]), sizeof(uint16_t));
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                const int64_t q = order[(size_t)p];
                const int64_t off = (int64_t)col[q] - i;
                const int32_t t = ntype ? ntype[q] : 0;
                if (off < -(int64_t(1) << 27) || off >= (int64_t(1) << 27)) {
                    ok = false;
                    break;
                }
                const int32_t e = (int32_t)((uint32_t)off << 4) | t;
                key.append(reinterpret_cast<const char*>(&e), sizeof(e));
            }
            if (!ok)
                break;
            auto it = ids.find(key);
            if (it == ids.end()) {
                const int id = (int)ids.size();
                const size_t cnt = (key.size() - sizeof(uint16_t)) / sizeof(int32_t);
                uint16_t nn;
                std::memcpy(&nn, key.data(), sizeof(nn));
                const size_t n_far = cnt - nn;
                lds_entries += cnt + (n_far < far_min ? far_min - n_far : 0);
                longest = std::max(longest, cnt);
                if (id >= kWideMaxPatterns || (size_t)(id + 1) * longest > (size_t)kWideMaxEntries) {
                    ok = false;
                    break;
                }
                it = ids.emplace(key, id).first;
                keys.push_back(key);
            }
            pid[(size_t)i] = (uint16_t)it->second;
        }
        auto entry = [&](const std::string& k, size_t c) {
            int32_t e;
            std::memcpy(&e, k.data() + sizeof(uint16_t) + c * sizeof(int32_t), sizeof(e));
            return e;
        };
        auto near_count = [&](const std::string& k) {
            uint16_t nn;
            std::memcpy(&nn, k.data(), sizeof(nn));
            return nn;
        };
        if (ok && keys.size() <= (size_t)kMaxPatterns && lds_entries <= (size_t)kMaxPatternEntries) {
            s.stencil = true;
            s.pat_id.resize((size_t)n);
            for (int64_t i = 0; i < n; ++i)
                s.pat_id[(size_t)i] = (uint8_t)pid[(size_t)i];
            s.pat_start.assign(1, 0);
            for (const std::string& k : keys) {
                const size_t cnt = (k.size() - sizeof(uint16_t)) / sizeof(int32_t);
                const uint16_t nn = near_count(k);
                s.pat_far.push_back((uint16_t)(s.pat_tab.size() + nn));
                for (size_t c = 0; c < cnt; ++c)
                    s.pat_tab.push_back(entry(k, c));
                const size_t n_far = cnt - nn;
                s.pat_tab.insert(s.pat_tab.end(), n_far < far_min ? far_min - n_far : 0, 0);
                s.pat_start.push_back((uint16_t)s.pat_tab.size());
            }
            s.no_far = !any_far;
            return s;
        }
        if (ok && !keys.empty()) {
            // entry c of pattern p at w_tab[c * patterns + p]; the near and
            // the far part of a pattern are each padded to whole batches,
            // and shorter patterns end in padding (type kMaxTypes, J = 0)
            const size_t np = keys.size();
            const int32_t pad = kMaxTypes;
            auto up = [](size_t c) { return (c + kWideBatch - 1) / kWideBatch * kWideBatch; };
            size_t len = 0;
            bool fits = true;
            for (const std::string& k : keys) {
                const size_t cnt = (k.size() - sizeof(uint16_t)) / sizeof(int32_t), nn = near_count(k);
                len = std::max(len, up(nn) + up(cnt - nn));
                for (size_t c = 0; c < cnt; ++c) {
                    const int32_t off = entry(k, c) >> 4;
                    fits = fits && off >= -(1 << 26) && off < (1 << 26);
                }
            }
            if (fits && len * np <= (size_t)kWideMaxEntries && len <= 0xFFFF) {
                s.wide = true;
                s.w_len = (int)len;
                s.w_pid = std::move(pid);
                s.w_tab.assign(len * np, pad);
                s.w_near.resize(np);
                for (size_t p = 0; p < np; ++p) {
                    const size_t cnt = (keys[p].size() - sizeof(uint16_t)) / sizeof(int32_t), nn = near_count(keys[p]);
                    s.w_near[p] = (uint16_t)up(nn);
                    for (size_t c = 0; c < cnt; ++c) {
                        const int32_t e = entry(keys[p], c);
                        const size_t slot = c < nn ? c : up(nn) + (c - nn);
                        s.w_tab[slot * np + p] = (int32_t)((uint32_t)(e >> 4) << 5) | (e & 15);
                    }
                }
                return s;
            }
        }
    }

    const int64_t n_slices = (n + kSlice - 1) / kSlice;
    s.slice_off.assign(n_slices + 1, 0);
    s.deg.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        s.deg[i] = ((uint32_t)n_near[(size_t)i] << 16) | (uint32_t)(row_ptr[i + 1] - row_ptr[i]);
        s.long_rows = s.long_rows || row_ptr[i + 1] - row_ptr[i] > kLongRow;
    }
    for (int64_t sl = 0; sl < n_slices; ++sl) {
        int width = 0;
        for (int64_t i = sl * kSlice; i < std::min<int64_t>(n, (sl + 1) * kSlice); ++i)
            width = std::max<int>(width, (int)(s.deg[i] & 0xFFFFu));
        s.slice_off[sl + 1] = s.slice_off[sl] + (int64_t)kSlice * width;
    }
    s.nb.assign((size_t)s.slice_off[n_slices], 0u);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t base = s.slice_off[i / kSlice] + (i % kSlice);
        int k = 0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p, ++k) {
            const int64_t q = order[(size_t)p];
            const uint32_t t = ntype ? ntype[q] : 0u;
            s.nb[(size_t)(base + (int64_t)k * kSlice)] = (t << kColBits) | (uint32_t)col[q];
        }
    }
    return s;
}

// The links of row i from the stored device form: (column, type) pairs.
template <typename F>
static void for_each_link(const HostStructure& s, int64_t i, F&& fn)
{
    if (s.stencil) {
        const int p = s.pat_id[(size_t)i];
        for (int e = s.pat_start[p]; e < s.pat_start[p + 1]; ++e) {
            const int32_t raw = s.pat_tab[(size_t)e];
            const int32_t off = raw >> 4;
            if (off != 0)   // offset 0: padding of the far part, never a link
                fn(i + off, raw & 15);
        }
        return;
    }
    if (s.wide) {
        const size_t np = s.w_near.size(), p = s.w_pid[(size_t)i];
        for (int e = 0; e < s.w_len; ++e) {
            const int32_t raw = s.w_tab[(size_t)e * np + p];
            if ((raw & 31) != kMaxTypes)   // type kMaxTypes: padding, never a link
                fn(i + (raw >> 5), raw & 31);
        }
        return;
    }
    const int64_t base = s.slice_off[(size_t)(i / kSlice)] + (i % kSlice);
    const int d = (int)(s.deg[(size_t)i] & 0xFFFFu);
    for (int k = 0; k < d; ++k) {
        const uint32_t e = s.nb[(size_t)(base + (int64_t)k * kSlice)];
        fn((int64_t)(e & kColMask), (int)(e >> kColBits));
    }
}

void set_lattice(HostStructure& s, int nb, const int cells[3], const int periodic[3])
{
    if (!cells || !periodic)
        fail(SLLG_E_ARG, "cells and periodic must not be NULL");
    if (nb < 1 || nb > 255 || cells[0] < 1 || cells[1] < 1 || cells[2] < 1)
        fail(SLLG_E_ARG, "need 1 <= n_basis <= 255 and at least one cell per axis");
    const int64_t n_cells = (int64_t)cells[0] * cells[1] * cells[2];
    if (n_cells * nb != s.n)
        fail(SLLG_E_ARG, "n_basis x cells = " + std::to_string(n_cells * nb) + " sites, the system has " +
                             std::to_string(s.n));
    HostLattice L;
    L.on = true;
    L.nb = nb;
    L.nx = cells[0];
    L.ny = cells[1];
    L.nz = cells[2];
    for (int a = 0; a < 3; ++a)
        L.per[a] = periodic[a] != 0;
    const int dim[3] = {L.nx, L.ny, L.nz};
    // offset of coordinate v from u on axis a: -1, 0 or +1, else 2
    auto delta = [&](int a, int64_t u, int64_t v) -> int {
        int64_t d = v - u;
        if (L.per[a]) {
            d = ((d % dim[a]) + dim[a]) % dim[a];
            if (d == 0) return 0;
            if (d == 1) return 1;
            if (d == dim[a] - 1) return -1;
            return 2;
        }
        return d >= -1 && d <= 1 ? (int)d : 2;
    };
    // one (plane, basis site) pattern from the plane's first site of that
    // basis; every other site of the plane must match it.  Planes are
    // split over host threads.
    std::vector<std::vector<FusedLink>> ref((size_t)L.nz * nb);
    const uint32_t unb = (uint32_t)nb, unx = (uint32_t)L.nx, uny = (uint32_t)L.ny;
    const int64_t plane_sites = (int64_t)nb * L.nx * L.ny;
    int n_threads = (int)std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
    n_threads = (int)std::min<int64_t>(n_threads, L.nz);
    std::vector<int64_t> bad_site((size_t)n_threads, -1);
    std::vector<char> uniform((size_t)n_threads, 1);
    auto work = [&](int w) {
        std::vector<FusedLink> row;
        for (int64_t z = (int64_t)L.nz * w / n_threads; z < (int64_t)L.nz * (w + 1) / n_threads; ++z) {
            for (int64_t i = z * plane_sites; i < (z + 1) * plane_sites; ++i) {
                const uint32_t c = (uint32_t)i / unb, b = (uint32_t)i % unb;
                const uint32_t x = c % unx, y = (c / unx) % uny;
                row.clear();
                bool bad = false;
                for_each_link(s, i, [&](int64_t j, int type) {
                    const uint32_t cj = (uint32_t)j / unb, t = cj / unx;
                    const int dx = delta(0, x, cj % unx), dy = delta(1, y, t % uny), dz = delta(2, z, t / uny);
                    bad = bad || dx == 2 || dy == 2 || dz == 2;
                    row.push_back(FusedLink{(int8_t)dz, (int8_t)dy, (int8_t)dx, (uint8_t)((uint32_t)j % unb),
                                            (uint8_t)type});
                });
                if (bad) {
                    bad_site[(size_t)w] = i;
                    return;
                }
                std::sort(row.begin(), row.end());
                std::vector<FusedLink>& r = ref[(size_t)z * nb + b];
                if (i - z * plane_sites < nb)
                    r = row;
                else if (uniform[(size_t)w] && row != r)
                    uniform[(size_t)w] = 0;
            }
        }
    };
    {
        std::vector<std::thread> pool;
        for (int w = 1; w < n_threads; ++w)
            pool.emplace_back(work, w);
        work(0);
        for (auto& th : pool)
            th.join();
    }
    for (int64_t i : bad_site)
        if (i >= 0)
            fail(SLLG_E_ARG, "site " + std::to_string(i) + " has a link to a cell more than one cell away "
                             "in the declared lattice");
    bool uniform_in_plane = true;
    for (char u : uniform)
        uniform_in_plane = uniform_in_plane && u;
    // patterns: distinct (basis site, link list)
    std::vector<uint8_t> plane(ref.size());
    bool by_basis = true;
    for (size_t key = 0; key < ref.size(); ++key) {
        const int b = (int)(key % nb);
        int id = -1;
        for (size_t p = 0; p < L.pats.size(); ++p)
            if (L.pat_b[p] == b && L.pats[p] == ref[key]) {
                id = (int)p;
                break;
            }
        if (id < 0) {
            if ((int)L.pats.size() >= kFusedMaxPatterns) {
                id = kFusedMaxPatterns;   // too many: not fusable (below)
            } else {
                id = (int)L.pats.size();
                L.pats.push_back(ref[key]);
                L.pat_b.push_back((uint8_t)b);
            }
        }
        plane[key] = (uint8_t)std::min(id, 255);
        by_basis = by_basis && id == b;
    }
    size_t entries = 0;
    for (const auto& p : L.pats)
        entries += p.size();
    if (!L.per[0] || !L.per[1])
        L.why = "the fused step needs periodic x and y";
    else if (nb > kFusedMaxBasis)
        L.why = "the fused step is built for at most " + std::to_string(kFusedMaxBasis) + " sites per cell";
    else if (!uniform_in_plane)
        L.why = "the links of a basis site change within a plane";
    else if ((int)L.pats.size() >= kFusedMaxPatterns || entries > (size_t)kFusedMaxEntries)
        L.why = "too many link patterns for the fused step";
    else if (L.nx > 0xFFFF || L.ny > 0xFFFF)
        L.why = "too many cells per axis for the fused step";
    L.fusable = L.why.empty();
    // a compiled kind: every (plane, basis site) has the kind's links, less
    // those into planes beyond an open z surface, with one type per slot
    for (int kind : {(int)kKindSc6, (int)kKindBcc8, (int)kKindBcc14}) {
        if (!L.fusable || kind_basis(kind) != nb)
            continue;
        int slot_type[2] = {-1, -1};
        bool match = true;
        for (int z = 0; z < L.nz && match; ++z)
            for (int b = 0; b < nb && match; ++b) {
                const std::vector<FusedLink>& have = ref[(size_t)z * nb + b];
                size_t k = 0;
                for (int dz = -1; dz <= 1 && match; ++dz) {
                    if (!L.per[2] && ((dz < 0 && z == 0) || (dz > 0 && z == L.nz - 1)))
                        continue;
                    for (int dy = -1; dy <= 1 && match; ++dy)
                        for (int dx = -1; dx <= 1 && match; ++dx)
                            for (int bp = 0; bp < nb && match; ++bp) {
                                int slot = 0;
                                if (!kind_link(kind, b, dz, dy, dx, bp, &slot))
                                    continue;
                                if (k >= have.size() || have[k].dz != dz || have[k].dy != dy || have[k].dx != dx ||
                                    have[k].bp != bp) {
                                    match = false;
                                    break;
                                }
                                if (slot_type[slot] < 0)
                                    slot_type[slot] = have[k].type;
                                match = slot_type[slot] == have[k].type;
                                ++k;
                            }
                }
                match = match && k == have.size();
            }
        if (match) {
            L.kind = kind;
            L.slot_type[0] = std::max(slot_type[0], 0);
            L.slot_type[1] = std::max(slot_type[1], 0);
            break;
        }
    }
    if (!by_basis)
        L.plane_pat = std::move(plane);
    s.lat = std::move(L);
}

void set_exchange_tensors(HostStructure& s, const double* Jt, int n_types)
{
    if (!Jt) {
        s.tensor = false;
        s.Jt.clear();
        return;
    }
    if (n_types != s.n_types)
        fail(SLLG_E_ARG, "exchange tensors: n_types must match the neighbour list's (" +
                             std::to_string(s.n_types) + ")");
    for (int q = 0; q < 9 * n_types; ++q)
        if (!std::isfinite(Jt[q]))
            fail(SLLG_E_ARG, "exchange tensor holds a non-finite value");
    if (s.rev_known)
        for (int t = 0; t < n_types; ++t)
            for (int u = 0; u < n_types; ++u)
                if (s.reverse[t] & (1u << u))
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            if (Jt[9 * u + 3 * b + a] != Jt[9 * t + 3 * a + b])
                                fail(SLLG_E_ARG, "exchange tensor of type " + std::to_string(u) +
                                                     " is not the transpose of type " + std::to_string(t) +
                                                     ", which its links reverse");
    s.Jt.assign(Jt, Jt + 9 * n_types);
    s.tensor = true;
}

HostDemag build_demag(int64_t n, const double* pos, double cell_size, double atom_volume, int64_t every)
{
    if (!pos)
        fail(SLLG_E_ARG, "positions must not be NULL");
    if (!(cell_size > 0.0) || !std::isfinite(cell_size) || !(atom_volume > 0.0) || !std::isfinite(atom_volume))
        fail(SLLG_E_ARG, "cell_size and atom_volume must be finite and > 0");
    if (every < 1)
        fail(SLLG_E_ARG, "every must be >= 1");
    HostDemag d;
    d.on = true;
    d.cell_size = cell_size;
    d.atom_volume = atom_volume;
    d.every = every;
    double lo[3] = {pos[0], pos[1], pos[2]}, hi[3] = {pos[0], pos[1], pos[2]};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            const double x = pos[3 * i + a];
            if (!std::isfinite(x))
                fail(SLLG_E_ARG, "positions must be finite");
            lo[a] = std::min(lo[a], x);
            hi[a] = std::max(hi[a], x);
        }
    for (int a = 0; a < 3; ++a)
        lo[a] -= cell_size / 1000.0;
    int64_t dims[3];
    for (int a = 0; a < 3; ++a) {
        const double ext = std::floor((hi[a] - lo[a]) / cell_size) + 1.0;
        if (ext > 2.0e6)
            fail(SLLG_E_ARG, "the sample spans too many macrocells along one axis");
        dims[a] = (int64_t)ext;
    }
    std::vector<std::pair<int64_t, int32_t>> key((size_t)n);
    d.pos.resize(3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (int64_t)std::floor((pos[3 * i + a] - lo[a]) / cell_size);
            d.pos[3 * i + a] = pos[3 * i + a] - lo[a];
        }
        key[(size_t)i] = {(c[0] * dims[1] + c[1]) * dims[2] + c[2], (int32_t)i};
    }
    std::sort(key.begin(), key.end());
    d.cell_of.resize((size_t)n);
    d.atoms.resize((size_t)n);
    d.start.assign(1, 0);
    for (int64_t k = 0; k < n; ++k) {
        if (k > 0 && key[(size_t)k].first != key[(size_t)k - 1].first)
            d.start.push_back((int32_t)k);
        d.cell_of[(size_t)key[(size_t)k].second] = (int32_t)d.start.size() - 1;
        d.atoms[(size_t)k] = key[(size_t)k].second;
    }
    d.start.push_back((int32_t)n);
    d.cells = (int64_t)d.start.size() - 1;
    return d;
}

void demag_cells(const HostDemag& dm, const HostMaterials& m, std::vector<double>& centre,
                 std::vector<double>& self)
{
    constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
    centre.assign(3 * (size_t)dm.cells, 0.0);
    self.assign((size_t)dm.cells, 0.0);
    for (int64_t p = 0; p < dm.cells; ++p) {
        double mu_sum = 0.0, x[3] = {0.0, 0.0, 0.0};
        for (int32_t k = dm.start[(size_t)p]; k < dm.start[(size_t)p + 1]; ++k) {
            const int32_t i = dm.atoms[(size_t)k];
            const double mu = m.mat_mu[m.per_site_material ? m.matid[(size_t)i] : 0];
            mu_sum += mu;
            for (int a = 0; a < 3; ++a)
                x[a] += mu * dm.pos[3 * (size_t)i + a];
        }
        for (int a = 0; a < 3; ++a)
            centre[3 * (size_t)p + a] = x[a] / mu_sum;
        const double atoms = (double)(dm.start[(size_t)p + 1] - dm.start[(size_t)p]);
        self[(size_t)p] = kMu0 / 3.0 / (atoms * dm.atom_volume);
    }
}

void build_colours(HostStructure& s, bool lattice_order)
{
    const int64_t n = s.n;
    // visiting order: ascending sites, or on a declared lattice the sites
    // of each basis site and cell parity (x + y + z even, then odd) in turn
    std::vector<int32_t> visit((size_t)n);   // site numbers fit 31 bits (colour_sites holds them as int32)
    const HostLattice& L = s.lat;
    if (lattice_order && L.on) {
        size_t v = 0;
        for (int b = 0; b < L.nb; ++b)
            for (int parity = 0; parity < 2; ++parity)
                for (int64_t i = b; i < n; i += L.nb) {
                    const int64_t cell = i / L.nb;
                    const int64_t x = cell % L.nx, y = (cell / L.nx) % L.ny, z = cell / ((int64_t)L.nx * L.ny);
                    if (((x + y + z) & 1) == parity)
                        visit[v++] = (int32_t)i;
                }
    } else {
        for (int64_t i = 0; i < n; ++i)
            visit[(size_t)i] = (int32_t)i;
    }
    // greedy: each site takes the smallest colour no earlier-visited
    // neighbour has (a site has at most kMaxDegree neighbours)
    std::vector<int32_t> colour((size_t)n, -1);
    std::vector<int64_t> seen(kMaxDegree + 2, -1);   // seen[c] == i: colour c is taken around site i
    int n_colours = 0;
    for (const int32_t vi : visit) {
        const int64_t i = vi;
        for_each_link(s, i, [&](int64_t j, int) {
            const int32_t cj = colour[(size_t)j];
            if (cj >= 0 && cj <= kMaxDegree)
                seen[(size_t)cj] = i;
        });
        int c = 0;
        while (seen[(size_t)c] == i)
            ++c;
        colour[(size_t)i] = c;
        n_colours = std::max(n_colours, c + 1);
    }
    s.colour_start.assign((size_t)n_colours + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        ++s.colour_start[(size_t)colour[(size_t)i] + 1];
    for (int c = 0; c < n_colours; ++c)
        s.colour_start[(size_t)c + 1] += s.colour_start[(size_t)c];
    std::vector<int64_t> fill(s.colour_start.begin(), s.colour_start.end() - 1);
    s.colour_sites.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        s.colour_sites[(size_t)fill[(size_t)colour[(size_t)i]]++] = (int32_t)i;
}

HostMaterials build_materials(int64_t n, const double* mu_s, const double* k_u,
                              const double* easy_axis, int per_site, const double* k_c, int kc_per_site)
{
    if (!mu_s || !k_u || !easy_axis)
        fail(SLLG_E_ARG, "mu_s, k_u and easy_axis must not be NULL");
    if (per_site != 0 && per_site != 1)
        fail(SLLG_E_ARG, "per_site must be 0 or 1");
    if (kc_per_site != 0 && kc_per_site != 1)
        fail(SLLG_E_ARG, "per_site must be 0 or 1");
    if (k_c)
        for (int64_t i = 0; i < (kc_per_site ? n : 1); ++i)
            if (!std::isfinite(k_c[i]))
                fail(SLLG_E_ARG, "k_c must be finite");
    const int64_t m = per_site ? n : 1;
    for (int64_t i = 0; i < m; ++i) {
        if (!(mu_s[i] > 0.0) || !std::isfinite(mu_s[i]))
            fail(SLLG_E_ARG, "mu_s must be positive and finite");
        if (!std::isfinite(k_u[i]))
            fail(SLLG_E_ARG, "k_u must be finite");
        const double* e = easy_axis + 3 * i;
        const double len = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        if (!(len > 0.0) || !std::isfinite(len))
            fail(SLLG_E_ARG, "easy axis of zero or non-finite length");
    }
    HostMaterials h;
    h.n = n;
    const bool kc_sites = k_c && kc_per_site;
    const int64_t mm = (per_site || kc_sites) ? n : 1;   // sites that may differ
    std::map<std::tuple<double, double, double>, int> ids;
    std::vector<uint8_t> matid(mm > 1 || per_site ? n : 0);
    for (int64_t i = 0; i < mm; ++i) {
        const double mu = mu_s[per_site ? i : 0], ku = k_u[per_site ? i : 0];
        const double kc = k_c ? k_c[kc_sites ? i : 0] : 0.0;
        auto key = std::make_tuple(mu, ku, kc);
        auto it = ids.find(key);
        int id;
        if (it == ids.end()) {
            id = (int)ids.size();
            if (id >= 256)
                fail(SLLG_E_ARG, "more than 256 distinct (mu_s, k_u, k_c) materials");
            ids.emplace(key, id);
            h.mat_mu.push_back(mu);
            h.mat_ku.push_back(ku);
            h.mat_kc.push_back(kc);
            h.cubic = h.cubic || kc != 0.0;
        } else {
            id = it->second;
        }
        if (!matid.empty())
            matid[i] = (uint8_t)id;
    }
    h.per_site_material = h.mat_mu.size() > 1;
    if (h.per_site_material)
        h.matid = std::move(matid);
    // easy axes
    auto unit = [&](int64_t i, double out[3]) {
        const double* e = easy_axis + 3 * i;
        const double len = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        out[0] = e[0] / len;
        out[1] = e[1] / len;
        out[2] = e[2] / len;
    };
    unit(0, h.axis);
    if (per_site) {
        for (int64_t i = 1; i < n && !h.per_site_axis; ++i) {
            const double* e = easy_axis + 3 * i;
            h.per_site_axis = e[0] != easy_axis[0] || e[1] != easy_axis[1] || e[2] != easy_axis[2];
        }
        if (h.per_site_axis) {
            h.axis_site.resize(3 * (size_t)n);
            for (int64_t i = 0; i < n; ++i)
                unit(i, &h.axis_site[3 * (size_t)i]);
        }
    }
    h.mu_ref = h.mat_mu[0];
    double tot = 0.0;
    if (per_site) {
        for (int64_t i = 0; i < n; ++i)
            tot += mu_s[i];
    } else {
        tot = mu_s[0] * (double)n;
    }
    h.mu_total = tot;
    return h;
}

std::vector<double> normalised_spins(int64_t n, const double* S, bool normalise)
{
    if (!S)
        fail(SLLG_E_ARG, "spin array must not be NULL");
    std::vector<double> out(3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const double* s = S + 3 * i;
        const double len = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        if (!(len > 0.0) || !std::isfinite(len))
            fail(SLLG_E_ARG, "spin " + std::to_string(i) + " has zero or non-finite length");
        out[3 * i] = normalise ? s[0] / len : s[0];
        out[3 * i + 1] = normalise ? s[1] / len : s[1];
        out[3 * i + 2] = normalise ? s[2] / len : s[2];
    }
    return out;
}

void check_dynamics(const Dynamics& d)
{
    if (!(d.alpha >= 0.0) || !std::isfinite(d.alpha))
        fail(SLLG_E_ARG, "damping must be finite and >= 0");
    if (!(d.gamma > 0.0) || !std::isfinite(d.gamma))
        fail(SLLG_E_ARG, "gamma must be finite and > 0");
    if (!(d.dt > 0.0) || !std::isfinite(d.dt))
        fail(SLLG_E_ARG, "dt must be finite and > 0");
    if (!(d.temperature >= 0.0) || !std::isfinite(d.temperature))
        fail(SLLG_E_ARG, "temperature must be finite and >= 0");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(d.H[c]))
            fail(SLLG_E_ARG, "applied field must be finite");
}

template <typename R>
std::vector<MaterialDev<R>> material_table(const HostMaterials& m, const Dynamics& d)
{
    std::vector<MaterialDev<R>> t(m.mat_mu.size());
    for (size_t q = 0; q < t.size(); ++q) {
        const double mu = m.mat_mu[q], ku = m.mat_ku[q];
        t[q].mu_rel = (R)(m.mu_ref / mu);
        t[q].mu_frac = (R)(mu / m.mu_ref);
        t[q].ani = (R)(2.0 * ku / mu);
        t[q].ku_mu = (R)(ku / mu);
        t[q].sigma = (R)std::sqrt(2.0 * d.alpha * kBoltzmann * d.temperature / (d.gamma * mu * d.dt));
        t[q].axis[0] = (R)m.axis[0];
        t[q].axis[1] = (R)m.axis[1];
        t[q].axis[2] = (R)m.axis[2];
        const double kc = q < m.mat_kc.size() ? m.mat_kc[q] : 0.0;
        t[q].cub = (R)(-2.0 * kc / mu);
        t[q].kc_mu = (R)(kc / mu);
        t[q].mu_s = mu;
    }
    return t;
}

template <typename R>
void fill_parameters(ReplicaDev<R>& rec, const HostStructure& s, const HostMaterials& m,
                     const Dynamics& d)
{
    for (int t = 0; t < kMaxTypes; ++t) {
        rec.jt[t] = t < s.n_types ? (R)(s.J[t] / m.mu_ref) : (R)0;
        for (int q = 0; q < 9; ++q)
            rec.jm[t][q] = s.tensor && t < s.n_types ? (R)(s.Jt[9 * t + q] / m.mu_ref) : (R)0;
    }
    rec.gdt = (R)(d.gamma / (1.0 + d.alpha * d.alpha) * d.dt);
    rec.alpha = (R)d.alpha;
    rec.H[0] = (R)d.H[0];
    rec.H[1] = (R)d.H[1];
    rec.H[2] = (R)d.H[2];
    rec.inv_mu_total = 1.0 / m.mu_total;
    rec.mu_ref = m.mu_ref;
    rec.seed = d.seed;
    rec.step = d.step;
    rec.n = (int32_t)s.n;
    rec.tile = tile_of(s, sizeof(R));
    rec.blocks = (int32_t)((s.n + rec.tile - 1) / rec.tile);
    rec.halo = s.halo;
    int32_t flags = rec.flags & (kRecord | kRecordSeries);
    if (m.per_site_material)
        flags |= kPerSiteMaterial;
    if (m.per_site_axis)
        flags |= kPerSiteAxis;
    if (s.stencil)
        flags |= kStencil;
    if (s.stencil && s.no_far)
        flags |= kNoFar;
    if (s.wide)
        flags |= kWide;
    if (s.tensor)
        flags |= kTensor;
    if (m.cubic)
        flags |= kCubic;
    if (s.demag.on)
        flags |= kDemag;
    if (!s.stencil && !s.wide && s.long_rows)
        flags |= kLongRows;
    // the fused step: a lattice it takes in this precision, uniform
    // materials, scalar exchange and no cubic anisotropy or demagnetising
    // field
    if (fused_precision_ok(s.lat, s.n, sizeof(R)) && !m.per_site_material && !m.per_site_axis && !s.tensor &&
        !m.cubic && !s.demag.on)
        flags |= kFused;
    rec.flags = flags;
    rec.f_nb = s.lat.nb;
    rec.f_nx = s.lat.nx;
    rec.f_ny = s.lat.ny;
    rec.f_nz = s.lat.nz;
    rec.f_zper = s.lat.per[2] ? 1 : 0;
    rec.f_npat = (int32_t)s.lat.pats.size();
    rec.f_kind = s.lat.kind;
    rec.f_pad = 0;
    for (int q = 0; q < 2; ++q)
        rec.f_kj[q] = s.lat.on ? rec.jt[s.lat.slot_type[q]] : (R)0;
    int32_t nent = 0;
    for (const auto& p : s.lat.pats)
        nent += (int32_t)p.size();
    rec.f_nent = nent;
    rec.n_patterns = s.stencil ? (int32_t)s.pat_start.size() - 1 : s.wide ? (int32_t)s.w_near.size() : 0;
    rec.w_len = s.wide ? s.w_len : 0;
    rec.dm_cells = s.demag.on ? (int32_t)s.demag.cells : 0;
    rec.dm_chunks = s.demag.on ? demag_chunks(s.demag.cells) : 0;
}

void averages_from_block_sums(const double* acc, int n_blocks, int64_t block_len, double out[8])
{
    double tot[5] = {0, 0, 0, 0, 0};
    for (int b = 0; b < n_blocks; ++b)
        for (int c = 0; c < 5; ++c)
            tot[c] += acc[5 * b + c];
    const double ns = (double)block_len * n_blocks;
    auto se = [&](int c) {
        if (n_blocks < 2)
            return std::nan("");
        const double mean = tot[c] / ns;
        double v = 0.0;
        for (int b = 0; b < n_blocks; ++b) {
            const double d = acc[5 * b + c] / (double)block_len - mean;
            v += d * d;
        }
        return std::sqrt(v / (n_blocks - 1) / n_blocks);
    };
    out[0] = tot[0] / ns;
    out[1] = se(0);
    out[2] = tot[1] / ns;
    out[3] = tot[2] / ns;
    out[4] = tot[3] / ns;
    out[5] = tot[4] / ns;
    out[6] = se(4);
    out[7] = (double)n_blocks;
}

template std::vector<MaterialDev<float>> material_table<float>(const HostMaterials&, const Dynamics&);
template std::vector<MaterialDev<double>> material_table<double>(const HostMaterials&, const Dynamics&);
template void fill_parameters<float>(ReplicaDev<float>&, const HostStructure&, const HostMaterials&,
                                     const Dynamics&);
template void fill_parameters<double>(ReplicaDev<double>&, const HostStructure&, const HostMaterials&,
                                      const Dynamics&);

}  // namespace sllg
