"""Crystal lattices and their neighbour lists (CSR), built on the host.

System generation follows the paper's appendix on atomistic system
generation: a unit cell is replicated on a grid in x, y and z, the crystal
is optionally cut to a shape, and the interaction list of every atom comes
from the neighbour template of its unit cell.  Here the interaction list is
stored in compressed-sparse-row form:

    row_ptr : int64 [n + 1]   entries of row i are row_ptr[i] .. row_ptr[i+1]-1
    col     : int32 [nnz]     neighbour site index, ascending within each row
    ntype   : uint8 [nnz]     interaction type, an index into a J table

Every link appears in both directions (j in row i and i in row j), with the
same type, which is how the exchange sum over i != j is written in the
section on the classical spin Hamiltonian.

This module only produces inputs (positions and neighbour lists).  It holds
no part of the spin dynamics and is shared by the oracle's tests, the GPU
tests and the benchmark.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Lattice",
    "simple_cubic",
    "sc_long_range",
    "bcc",
    "fcc_sphere",
    "fcc_ellipsoid",
    "csr_from_padded",
]


class Lattice:
    """Positions (in units of the cubic cell edge a) plus a CSR neighbour list."""

    def __init__(self, kind, pos, row_ptr, col, ntype, dims=None, periodic=None):
        self.kind = kind
        self.pos = pos                      # float64 [n, 3], units of a
        self.row_ptr = row_ptr              # int64 [n + 1]
        self.col = col                      # int32 [nnz]
        self.ntype = ntype                  # uint8 [nnz]
        self.dims = dims                    # cells per axis (None for cut shapes)
        self.periodic = periodic            # tuple of bools (None for cut shapes)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def csr_from_padded(nbr: np.ndarray, typ: np.ndarray):
    """Turn a padded neighbour table (-1 = no neighbour) into sorted CSR rows."""
    n, k = nbr.shape
    # one sort key per entry: column in the high bits, type in the low 8 bits
    kdt = np.int32 if n < (1 << 23) else np.int64
    big = np.iinfo(kdt).max
    key = nbr.astype(kdt)
    key <<= 8
    key |= typ.astype(kdt)
    full = bool((nbr >= 0).all())
    if not full:
        key[nbr < 0] = big
    key.sort(axis=1)
    if full:
        deg = np.full(n, k, dtype=np.int64)
        flat = key.reshape(-1)
    else:
        valid = key != big
        deg = valid.sum(axis=1).astype(np.int64)
        flat = key[valid]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    ntype = (flat & 0xFF).astype(np.uint8)
    flat >>= 8
    col = flat.astype(np.int32, copy=False)
    return row_ptr, col, ntype


def _cell_grid(dims):
    lx, ly, lz = dims
    z, y, x = np.meshgrid(np.arange(lz, dtype=np.int32), np.arange(ly, dtype=np.int32),
                          np.arange(lx, dtype=np.int32), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def _wrap(c, length, periodic):
    """Wrap a cell coordinate; returns (coord, valid)."""
    if periodic:
        return np.mod(c, length), np.ones(c.shape, dtype=bool)
    return c, (c >= 0) & (c < length)


def simple_cubic(dims, periodic=(True, True, True)) -> Lattice:
    """Simple-cubic lattice, one site per cell, 6 nearest neighbours.

    Site index i = x + Lx * (y + Ly * z).
    """
    dims = tuple(int(d) for d in (dims if np.ndim(dims) else (dims,) * 3))
    lx, ly, lz = dims
    for length, p in zip(dims, periodic):
        if p and length < 3:
            raise ValueError("a periodic axis needs at least 3 cells")
    x, y, z = _cell_grid(dims)
    n = x.size
    offsets = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    nbr = np.full((n, 6), -1, dtype=np.int32)
    for k, (dx, dy, dz) in enumerate(offsets):
        nx, vx = _wrap(x + dx, lx, periodic[0])
        ny, vy = _wrap(y + dy, ly, periodic[1])
        nz, vz = _wrap(z + dz, lz, periodic[2])
        ok = vx & vy & vz
        nbr[ok, k] = (nx + lx * (ny + ly * nz))[ok]
    typ = np.zeros((n, 6), dtype=np.uint8)
    row_ptr, col, ntype = csr_from_padded(nbr, typ)
    pos = np.stack([x, y, z], axis=1).astype(np.float64)
    return Lattice("sc", pos, row_ptr, col, ntype, dims, tuple(periodic))


def sc_long_range(L, r_cut, n_types=16):
    """Periodic simple-cubic L^3 lattice in which every site is linked to all
    sites within r_cut lattice constants (hundreds of partners for r_cut
    around 4).  The distances are cut into at most n_types bins of equal
    width in r (type t covers 1 + t (r_cut - 1)/n_types .. the next bound);
    shells() returns the (r_lo, r_hi) of every type.  L must exceed 2 r_cut
    so that no pair is linked twice through the periodic images."""
    if L <= 2 * r_cut:
        raise ValueError("L must exceed 2 r_cut")
    m = int(np.floor(r_cut))
    rng_ = np.arange(-m, m + 1)
    dz, dy, dx = np.meshgrid(rng_, rng_, rng_, indexing="ij")
    off = np.stack([dx.ravel(), dy.ravel(), dz.ravel()], axis=1)
    r = np.sqrt((off ** 2).sum(1))
    keep = (r > 0) & (r <= r_cut + 1e-9)
    off, r = off[keep], r[keep]
    edges = 1.0 + (r_cut - 1.0) * np.arange(n_types + 1) / n_types
    edges[-1] = r_cut + 1e-6
    typ = np.clip(np.searchsorted(edges, r, side="right") - 1, 0, n_types - 1).astype(np.uint8)
    x, y, z = _cell_grid((L, L, L))
    n = x.size
    nbr = np.empty((n, off.shape[0]), dtype=np.int32)
    for k, (ox, oy, oz) in enumerate(off):
        nbr[:, k] = ((x + ox) % L) + L * (((y + oy) % L) + L * ((z + oz) % L))
    row_ptr, col, ntype = csr_from_padded(nbr, np.tile(typ, (n, 1)))
    pos = np.stack([x, y, z], axis=1).astype(np.float64)
    lat = Lattice("sc", pos, row_ptr, col, ntype, (L, L, L), (True, True, True))
    lat.shells = [(edges[t], edges[t + 1]) for t in range(n_types)]
    return lat


def bcc(dims, periodic=(True, True, True), second_neighbours=False) -> Lattice:
    """Body-centred-cubic lattice, two sites per cell.

    Basis (0,0,0) (s = 0) and (1/2,1/2,1/2) (s = 1); site index
    i = 2 * (x + Lx * (y + Ly * z)) + s.  First neighbours (type 0) sit at
    a*sqrt(3)/2: 8 per site.  With ``second_neighbours`` the 6 sites at
    distance a (same sublattice, one cell along each axis) are added as
    type 1.
    """
    dims = tuple(int(d) for d in (dims if np.ndim(dims) else (dims,) * 3))
    lx, ly, lz = dims
    for length, p in zip(dims, periodic):
        if p and length < 3:
            raise ValueError("a periodic axis needs at least 3 cells")
    x, y, z = _cell_grid(dims)
    ncell = x.size
    k_max = 14 if second_neighbours else 8
    nbr = np.full((ncell, 2, k_max), -1, dtype=np.int32)
    typ = np.zeros((ncell, 2, k_max), dtype=np.uint8)

    def site_index(cx, cy, cz, s):
        return 2 * (cx + lx * (cy + ly * cz)) + s

    corner = [(dx, dy, dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
    for s in (0, 1):
        k = 0
        # s = 0 at cell c touches the body centres of cells c + {-1, 0}^3;
        # s = 1 at cell c touches the corners of cells c + {0, 1}^3.
        for (dx, dy, dz) in corner:
            if s == 0:
                dx, dy, dz = dx - 1, dy - 1, dz - 1
            nx, vx = _wrap(x + dx, lx, periodic[0])
            ny, vy = _wrap(y + dy, ly, periodic[1])
            nz, vz = _wrap(z + dz, lz, periodic[2])
            ok = vx & vy & vz
            nbr[ok, s, k] = site_index(nx, ny, nz, 1 - s)[ok]
            k += 1
        if second_neighbours:
            for (dx, dy, dz) in [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]:
                nx, vx = _wrap(x + dx, lx, periodic[0])
                ny, vy = _wrap(y + dy, ly, periodic[1])
                nz, vz = _wrap(z + dz, lz, periodic[2])
                ok = vx & vy & vz
                nbr[ok, s, k] = site_index(nx, ny, nz, s)[ok]
                typ[:, s, k] = 1
                k += 1
    nbr = nbr.reshape(2 * ncell, k_max)
    typ = typ.reshape(2 * ncell, k_max)
    row_ptr, col, ntype = csr_from_padded(nbr, typ)
    pos = np.empty((2 * ncell, 3), dtype=np.float64)
    base = np.stack([x, y, z], axis=1).astype(np.float64)
    pos[0::2] = base
    pos[1::2] = base + 0.5
    return Lattice("bcc", pos, row_ptr, col, ntype, dims, tuple(periodic))


def fcc_ellipsoid(a_nm: float, semi_axes_nm, tie: float = 1e-9) -> Lattice:
    """Ellipsoid cut from an fcc crystal, centred on a lattice site: the sites
    (x, y, z) * a/2 (x + y + z even) with sum_k (x_k / r_k)^2 <= 1 + tie for
    semi-axes r = semi_axes_nm along x, y, z.  Nearest neighbours as in
    fcc_sphere; positions in units of a."""
    half = a_nm / 2.0
    r = np.asarray(semi_axes_nm, dtype=np.float64)
    m = int(np.floor(r.max() / half)) + 1
    rng = np.arange(-m, m + 1)
    z, y, x = np.meshgrid(rng, rng, rng, indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    q = (x * half / r[0]) ** 2 + (y * half / r[1]) ** 2 + (z * half / r[2]) ** 2
    keep = ((x + y + z) % 2 == 0) & (q <= 1.0 + tie)
    return _fcc_from_points(x[keep], y[keep], z[keep], m, "fcc_ellipsoid")


def _fcc_from_points(x, y, z, m, kind):
    n = x.size
    width = 2 * m + 1
    grid = np.full((width, width, width), -1, dtype=np.int64)
    grid[z + m, y + m, x + m] = np.arange(n)
    offsets = [(sx, sy, 0) for sx in (-1, 1) for sy in (-1, 1)] + \
              [(sx, 0, sz) for sx in (-1, 1) for sz in (-1, 1)] + \
              [(0, sy, sz) for sy in (-1, 1) for sz in (-1, 1)]
    nbr = np.full((n, 12), -1, dtype=np.int64)
    for k, (dx, dy, dz) in enumerate(offsets):
        nx, ny, nz = x + dx + m, y + dy + m, z + dz + m
        inside = (nx >= 0) & (nx < width) & (ny >= 0) & (ny < width) & (nz >= 0) & (nz < width)
        j = np.full(n, -1, dtype=np.int64)
        j[inside] = grid[nz[inside], ny[inside], nx[inside]]
        nbr[:, k] = j
    typ = np.zeros((n, 12), dtype=np.uint8)
    row_ptr, col, ntype = csr_from_padded(nbr, typ)
    pos = np.stack([x, y, z], axis=1).astype(np.float64) * 0.5
    return Lattice(kind, pos, row_ptr, col, ntype, None, None)


def fcc_sphere(a_nm: float, radius_nm: float, tie_nm: float = 1e-9) -> Lattice:
    """Sphere cut from an fcc crystal, centred on a lattice site.

    Sites are the points (x, y, z) * a/2 with integer x + y + z even; a site
    belongs to the particle if its distance from the centre is at most
    ``radius_nm + tie_nm``.  Nearest neighbours (type 0) sit at a/sqrt(2),
    12 in the bulk and fewer at the surface.  Site order is z-major, then y,
    then x.  Positions are returned in units of a.
    """
    half = a_nm / 2.0
    r_half = (radius_nm + tie_nm) / half
    m = int(np.floor(r_half)) + 1
    rng = np.arange(-m, m + 1)
    z, y, x = np.meshgrid(rng, rng, rng, indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    keep = ((x + y + z) % 2 == 0) & (
        (x.astype(np.float64) ** 2 + y ** 2 + z ** 2) * half * half <= (radius_nm + tie_nm) ** 2
    )
    x, y, z = x[keep], y[keep], z[keep]
    n = x.size
    width = 2 * m + 1
    grid = np.full((width, width, width), -1, dtype=np.int64)
    grid[z + m, y + m, x + m] = np.arange(n)
    offsets = [(sx, sy, 0) for sx in (-1, 1) for sy in (-1, 1)] + \
              [(sx, 0, sz) for sx in (-1, 1) for sz in (-1, 1)] + \
              [(0, sy, sz) for sy in (-1, 1) for sz in (-1, 1)]
    nbr = np.full((n, 12), -1, dtype=np.int64)
    for k, (dx, dy, dz) in enumerate(offsets):
        nx, ny, nz = x + dx + m, y + dy + m, z + dz + m
        inside = (nx >= 0) & (nx < width) & (ny >= 0) & (ny < width) & (nz >= 0) & (nz < width)
        j = np.full(n, -1, dtype=np.int64)
        j[inside] = grid[nz[inside], ny[inside], nx[inside]]
        nbr[:, k] = j
    typ = np.zeros((n, 12), dtype=np.uint8)
    row_ptr, col, ntype = csr_from_padded(nbr, typ)
    pos = np.stack([x, y, z], axis=1).astype(np.float64) * 0.5
    return Lattice("fcc_sphere", pos, row_ptr, col, ntype, None, None)
