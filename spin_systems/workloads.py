"""Synthetic workloads shaped like the systems the paper simulates.

Material constants come from Table 1 (Bohr magneton, gyromagnetic ratio)
and Table 2 (bcc Fe: a = 2.866 A, mu_s = 2.22 muB, J = 7.05e-21 J/link,
k = 5.65e-25 J/atom; fcc Ni: a = 3.524 A, J = 2.757e-21 J/link,
k = 5.47e-26 J/atom).  The simple-cubic material (J = 6.0e-21 J/link) is the
test system of the Monte Carlo vs LLG comparison in the section on Monte
Carlo methods.

Every random draw here is seeded; nothing in this module integrates spins.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lattice import Lattice, bcc, fcc_sphere, sc_long_range, simple_cubic

MU_B = 9.2740e-24      # J/T, Table 1
GAMMA = 1.76e11        # 1/(T s), Table 1

__all__ = [
    "MU_B", "GAMMA", "Workload",
    "sc_reference", "bcc_film", "fcc_nanoparticle", "bcc_block", "serving_requests",
    "sc_request_system", "single_spin", "dmi_matrix", "with_tensor_exchange", "with_demag",
    "long_range_sc",
]


@dataclass
class Workload:
    """One spin system plus its integration settings (SI units)."""
    name: str
    lattice: Lattice
    J: np.ndarray                    # J per interaction type, joules/link
    mu_s: np.ndarray                 # [n] J/T
    k_u: np.ndarray                  # [n] J/atom
    easy_axis: np.ndarray            # [n, 3] unit vectors
    alpha: float
    gamma: float
    dt: float
    temperature: float
    H: np.ndarray                    # [3] tesla
    seed: int
    n_steps: int
    S0: np.ndarray                   # [n, 3] unit vectors
    extra: dict = field(default_factory=dict)
    J_tensor: np.ndarray | None = None   # [n_types, 3, 3] joules/link, replaces J when set
    k_c: np.ndarray | None = None        # [n] cubic anisotropy, J/atom
    demag: dict | None = None            # macrocell demagnetising field (with_demag)

    @property
    def n(self) -> int:
        return self.lattice.n

    def uniform_materials(self) -> bool:
        return bool(np.all(self.mu_s == self.mu_s[0]) and np.all(self.k_u == self.k_u[0])
                    and np.all(self.easy_axis == self.easy_axis[0]))


def _uniform(n, value):
    return np.full(n, float(value), dtype=np.float64)


def _axis(n, vec=(0.0, 0.0, 1.0)):
    return np.tile(np.asarray(vec, dtype=np.float64), (n, 1))


def _spins(n, direction):
    return _axis(n, direction)


def sc_reference(L=16, temperature=300.0, n_steps=1000, seed=42, alpha=0.1, dt=1e-16) -> Workload:
    """Simple-cubic ferromagnet, periodic, 6 neighbours, J = 6.0e-21 J/link,
    mu_s = 1.5 muB, k_u = 1e-23 J along z, no applied field, spins along +z.
    At L = 16 this is the 4096-spin reference system."""
    lat = simple_cubic(L, (True, True, True))
    n = lat.n
    return Workload(
        name=f"sc{L}^3", lattice=lat, J=np.array([6.0e-21]),
        mu_s=_uniform(n, 1.5 * MU_B), k_u=_uniform(n, 1.0e-23), easy_axis=_axis(n),
        alpha=alpha, gamma=GAMMA, dt=dt, temperature=temperature,
        H=np.zeros(3), seed=seed, n_steps=n_steps, S0=_spins(n, (0, 0, 1)))


def bcc_film(nx=64, ny=64, nz=16, seed=1, alpha=1.0, dt=1e-16) -> Workload:
    """bcc Fe-like film: periodic in x and y, open in z, 8 first neighbours
    (4 on the two surfaces), J = 7.05e-21, mu_s = 2.22 muB, k_u = 5.65e-25 J
    along z.  The temperature ramp runs 0..1500 K in 50 K steps with
    5000 equilibration plus 5000 averaging steps per point."""
    lat = bcc((nx, ny, nz), (True, True, False))
    n = lat.n
    temps = np.arange(0.0, 1500.0 + 1e-9, 50.0)
    return Workload(
        name=f"bcc film {nx}x{ny}x{nz}", lattice=lat, J=np.array([7.05e-21]),
        mu_s=_uniform(n, 2.22 * MU_B), k_u=_uniform(n, 5.65e-25), easy_axis=_axis(n),
        alpha=alpha, gamma=GAMMA, dt=dt, temperature=0.0, H=np.zeros(3), seed=seed,
        n_steps=5000, S0=_spins(n, (0, 0, 1)),
        extra={"temperatures": temps, "n_eq": 5000, "n_avg": 5000})


def fcc_nanoparticle(radius_nm=8.0, a_nm=0.3524, seed=2, axis_seed=2, alpha=0.1, dt=1e-16,
                     temperature=10.0) -> Workload:
    """Spherical fcc Ni-like particle cut from a lattice with a = 0.3524 nm.

    12 nearest neighbours in the core, fewer at the surface (a ragged CSR).
    J = 2.757e-21, mu_s = 0.6 muB.  Core sites: k_u = 5.47e-26 J along z.
    Surface sites (coordination < 12): k_u = 1e-23 J along a random axis drawn
    uniformly on the sphere (a normalised 3D Gaussian vector, the same
    construction as the uniform trial move of the Monte Carlo section).
    The field sweep runs from -5 T to +5 T along z in 0.1 T steps, 2000 steps
    per point; spins start along -z (along the first field)."""
    lat = fcc_sphere(a_nm, radius_nm)
    n = lat.n
    deg = lat.degree()
    surface = deg < 12
    k_u = np.where(surface, 1.0e-23, 5.47e-26)
    axes = _axis(n)
    rng = np.random.default_rng(axis_seed)
    g = rng.standard_normal((int(surface.sum()), 3))
    axes[surface] = g / np.linalg.norm(g, axis=1, keepdims=True)
    fields = np.round(np.arange(-50, 51) * 0.1, 10)
    return Workload(
        name=f"fcc sphere R={radius_nm}nm", lattice=lat, J=np.array([2.757e-21]),
        mu_s=_uniform(n, 0.6 * MU_B), k_u=k_u.astype(np.float64), easy_axis=axes,
        alpha=alpha, gamma=GAMMA, dt=dt, temperature=temperature,
        H=np.array([0.0, 0.0, -5.0]), seed=seed, n_steps=2000, S0=_spins(n, (0, 0, -1)),
        extra={"fields_z": fields, "steps_per_point": 2000, "surface": surface})


def bcc_block(cells=160, seed=4, alpha=0.05, dt=1e-16, temperature=300.0, n_steps=10000) -> Workload:
    """Periodic bcc block with first (J1 = 7.05e-21 J, 8 per site) and second
    (J2 = 3.0e-21 J, 6 per site) neighbours: 14 entries per CSR row.
    mu_s = 2.22 muB, k_u = 5.65e-25 J along z, spins start along +z.
    At 160 cells per edge this is 8,192,000 spins."""
    lat = bcc((cells,) * 3, (True, True, True), second_neighbours=True)
    n = lat.n
    return Workload(
        name=f"bcc {cells}^3 J1+J2", lattice=lat, J=np.array([7.05e-21, 3.0e-21]),
        mu_s=_uniform(n, 2.22 * MU_B), k_u=_uniform(n, 5.65e-25), easy_axis=_axis(n),
        alpha=alpha, gamma=GAMMA, dt=dt, temperature=temperature, H=np.zeros(3),
        seed=seed, n_steps=n_steps, S0=_spins(n, (0, 0, 1)))


def sc_request_system(L, temperature, H, n_steps, seed) -> Workload:
    """One serving request: periodic simple-cubic L^3 with the 4096-spin
    reference system's materials, alpha = 0.1, dt = 1e-16 s, spins along +z."""
    w = sc_reference(L=L, temperature=temperature, n_steps=n_steps, seed=seed)
    w.H = np.asarray(H, dtype=np.float64)
    w.name = f"request sc{L}^3"
    return w


def serving_requests(n_requests=512, rate_hz=200.0, seed=3, L_range=(8, 48),
                     T_range=(0.0, 1200.0), H_max=2.0, steps_range=(2000, 20000),
                     seed_base=1000):
    """Poisson arrivals of independent requests (a list of dicts).

    Inter-arrival times are exponential with mean 1/rate; L is uniform on
    the integers L_range; T uniform on T_range; |H| uniform on [0, H_max]
    along a direction uniform on the sphere; the step count uniform on the
    integers steps_range; request k uses RNG seed seed_base + k."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    Ls = rng.integers(L_range[0], L_range[1] + 1, size=n_requests)
    Ts = rng.uniform(T_range[0], T_range[1], size=n_requests)
    hmag = rng.uniform(0.0, H_max, size=n_requests)
    d = rng.standard_normal((n_requests, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    steps = rng.integers(steps_range[0], steps_range[1] + 1, size=n_requests)
    out = []
    for k in range(n_requests):
        out.append({
            "id": k, "arrival_s": float(arrivals[k]), "L": int(Ls[k]),
            "temperature": float(Ts[k]), "H": (hmag[k] * d[k]).tolist(),
            "n_steps": int(steps[k]), "seed": seed_base + k,
        })
    return out


def single_spin(mu_s=1.5 * MU_B, k_u=0.0, axis=(0.0, 0.0, 1.0), H=(0.0, 0.0, 0.0), alpha=0.1,
                dt=1e-15, temperature=0.0, S0=(1.0, 0.0, 0.0), seed=0, n_steps=1000) -> Workload:
    """An isolated spin (no neighbours), as in the paper's single-spin tests."""
    from .lattice import Lattice as _L
    lat = _L("single", np.zeros((1, 3)), np.zeros(2, dtype=np.int64),
             np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.uint8))
    s0 = np.asarray(S0, dtype=np.float64)
    s0 = s0 / np.linalg.norm(s0)
    ax = np.asarray(axis, dtype=np.float64)
    ax = ax / np.linalg.norm(ax)
    return Workload(
        name="single spin", lattice=lat, J=np.array([0.0]),
        mu_s=np.array([float(mu_s)]), k_u=np.array([float(k_u)]), easy_axis=ax[None, :],
        alpha=alpha, gamma=GAMMA, dt=dt, temperature=temperature,
        H=np.asarray(H, dtype=np.float64), seed=seed, n_steps=n_steps, S0=s0[None, :])


def dmi_matrix(D):
    """The matrix A with S_i^T A S_j = D . (S_i x S_j)."""
    Dx, Dy, Dz = (float(v) for v in D)
    return np.array([[0.0, Dz, -Dy], [-Dz, 0.0, Dx], [Dy, -Dx, 0.0]])


def with_tensor_exchange(w, D=0.0, dmi="bulk", k_c=None) -> Workload:
    """A copy of a periodic-lattice workload with one interaction type per
    (shell, bond direction) and exchange tensors J_ij = J_shell I - A(D_ij):
    the isotropic exchange of w plus a Dzyaloshinskii-Moriya energy
    D_ij . (S_i x S_j) per link, D_ij = D r_ij ("bulk") or D (z x r_ij)
    ("interfacial") with r_ij the unit bond vector (D in joules, one value
    or one per shell).  The reverse link gets the transposed tensor.  k_c
    (one value or [n], J/atom) adds cubic anisotropy."""
    lat = w.lattice
    n = lat.n
    p2 = np.rint(lat.pos * 2.0).astype(np.int32)          # positions in units of a/2
    if not np.allclose(p2, lat.pos * 2.0):
        raise ValueError("positions are not on the a/2 grid of the builders")
    rows = np.repeat(np.arange(n, dtype=np.intp), np.diff(lat.row_ptr))
    cols = lat.col.astype(np.intp)
    key = lat.ntype.astype(np.int32) * 125
    for a, scale in enumerate((25, 5, 1)):
        pa = np.ascontiguousarray(p2[:, a])
        q = pa[cols]
        q -= pa[rows]
        if lat.dims is not None and lat.periodic[a]:
            L2 = 2 * int(lat.dims[a])                      # minimum image
            q[q > L2 // 2] -= L2
            q[q < -(L2 // 2)] += L2
        if np.abs(q).max(initial=0) > 2:
            raise ValueError("bond vectors longer than the a/2 grid of the builders allows")
        key += (q + 2) * scale
    present = np.zeros(16 * 125, dtype=bool)
    present[key] = True
    uniq = np.nonzero(present)[0]
    if uniq.size > 16:
        raise ValueError(f"{uniq.size} directed interaction types (at most 16)")
    new_type = (np.cumsum(present) - 1).astype(np.uint8)[key]
    shells = uniq // 125
    vec = np.stack([(uniq // 25) % 5 - 2, (uniq // 5) % 5 - 2, uniq % 5 - 2], axis=1).astype(np.float64)
    rhat = vec / np.linalg.norm(vec, axis=1, keepdims=True)
    Dsh = np.broadcast_to(np.asarray(D, dtype=np.float64), (int(shells.max()) + 1,))
    J_iso = np.asarray(w.J, dtype=np.float64)[shells]
    tens = np.empty((uniq.size, 3, 3))
    for t in range(uniq.size):
        Dvec = Dsh[shells[t]] * (rhat[t] if dmi == "bulk" else np.cross([0.0, 0.0, 1.0], rhat[t]))
        tens[t] = J_iso[t] * np.eye(3) - dmi_matrix(Dvec)
    new_lat = Lattice(lat.kind + " directed", lat.pos, lat.row_ptr, lat.col, new_type, lat.dims,
                      lat.periodic)
    out = Workload(name=w.name + f" + DMI {dmi}", lattice=new_lat, J=J_iso, mu_s=w.mu_s, k_u=w.k_u,
                   easy_axis=w.easy_axis, alpha=w.alpha, gamma=w.gamma, dt=w.dt,
                   temperature=w.temperature, H=w.H, seed=w.seed, n_steps=w.n_steps, S0=w.S0,
                   extra=dict(w.extra), J_tensor=tens)
    if k_c is not None:
        out.k_c = np.ascontiguousarray(np.broadcast_to(np.asarray(k_c, dtype=np.float64), (n,)))
    return out


ATOMS_PER_CELL = {"sc": 1, "bcc": 2, "fcc_sphere": 4, "fcc_ellipsoid": 4}


def with_demag(w, a_nm, cell_size_nm, every=100, atom_volume_nm3=None) -> Workload:
    """w with the macrocell demagnetising field switched on: atom positions in
    metres (lattice positions times the cubic cell edge a_nm), macrocells of
    edge cell_size_nm, updated every `every` steps; the atomic volume
    defaults to a^3 / (atoms per cubic cell)."""
    if atom_volume_nm3 is None:
        kind = w.lattice.kind.split(" ")[0]
        atom_volume_nm3 = a_nm ** 3 / ATOMS_PER_CELL[kind]
    w.demag = {"pos": np.ascontiguousarray(w.lattice.pos * (a_nm * 1e-9)), "cell_size": cell_size_nm * 1e-9,
               "atom_volume": atom_volume_nm3 * 1e-27, "every": int(every)}
    return w


def long_range_sc(L=16, r_cut=4.5, J1=6.0e-21, decay=1.0, temperature=300.0, seed=5, n_steps=1000,
                  alpha=0.1, dt=1e-16) -> Workload:
    """Long-range exchange on a periodic simple-cubic lattice (the paper's
    remark that exchange can reach hundreds of partners): every pair within
    r_cut lattice constants is linked, J(r) = J1 exp(-(r - 1)/decay) taken
    at the middle of each of 16 radial bins.  At r_cut = 4.5, 388 partners
    per site.  Materials and start as the simple-cubic test system."""
    lat = sc_long_range(L, r_cut)
    mid = np.array([0.5 * (a + b) for a, b in lat.shells])
    J = J1 * np.exp(-(mid - 1.0) / decay)
    n = lat.n
    return Workload(
        name=f"sc {L}^3 long-range r<={r_cut}", lattice=lat, J=J, mu_s=_uniform(n, 1.5 * MU_B),
        k_u=_uniform(n, 1e-23), easy_axis=_axis(n), alpha=alpha, gamma=GAMMA, dt=dt,
        temperature=temperature, H=np.zeros(3), seed=seed, n_steps=n_steps, S0=_spins(n, (0, 0, 1)))
