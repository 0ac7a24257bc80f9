"""FP64 CPU oracle for the Heun-integrated stochastic LLG spin model.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the GPU library
never loads or calls it.  The arithmetic lives in plain C (``llg.c``,
``philox.c``), compiled with ``-O2 -ffp-contract=off`` and run on one
thread.  This module compiles that C, marshals numpy arrays into it, and
adds the statistics the paper's sweep protocols need (means and blocked
standard errors), written in numpy.

Paper passages: the section on the classical spin Hamiltonian (energy),
"Spin Dynamics" and "Langevin Dynamics" (LLG and thermal field), "Time
Integration of the LLG Equation" (Heun scheme), "Monte Carlo Methods"
(Metropolis acceptance with Hinzke-Nowak trial moves, ``mc.c``), the temperature-dependent
magnetisation protocol of the "Curie temperature" test (heating with the
previous state as the next starting point), and the Stoner-Wohlfarth test
(relaxation until the torque falls below 1e-6 T).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["philox.c", "llg.c", "mc.c", "demag.c"]
KB = 1.3807e-23  # J/K, Table 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C into ``oracle/liboracle.so`` (gcc, -O2, no FMA contraction)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall", "-Wextra",
           "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Demag(ctypes.Structure):
    _fields_ = [
        ("pos", ctypes.c_void_p),
        ("cell_size", ctypes.c_double),
        ("atom_volume", ctypes.c_double),
        ("every", ctypes.c_int64),
        ("field", ctypes.c_void_p),
        ("valid", ctypes.c_int),
        ("n_cells", ctypes.c_int64),
    ]


class _System(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("ntype", ctypes.c_void_p),
        ("J", ctypes.c_void_p),
        ("n_types", ctypes.c_int),
        ("mu_s", ctypes.c_void_p),
        ("k_u", ctypes.c_void_p),
        ("easy_axis", ctypes.c_void_p),
        ("alpha", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("temperature", ctypes.c_double),
        ("H", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64),
        ("J_tensor", ctypes.c_void_p),
        ("k_c", ctypes.c_void_p),
        ("demag", ctypes.POINTER(_Demag)),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.orc_philox_batch.argtypes = [ctypes.c_int64, P, P, P]
        L.orc_gaussian3_batch.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P,
                                          ctypes.c_uint32, P]
        L.orc_effective_fields.argtypes = [ctypes.POINTER(_System), P, P]
        L.orc_energy.argtypes = [ctypes.POINTER(_System), P]
        L.orc_energy.restype = ctypes.c_double
        L.orc_magnetisation.argtypes = [ctypes.POINTER(_System), P, P]
        L.orc_integrate.argtypes = [ctypes.POINTER(_System), P, ctypes.c_uint64, ctypes.c_int64, P, P]
        L.orc_integrate.restype = ctypes.c_int
        L.orc_relax.argtypes = [ctypes.POINTER(_System), P, ctypes.c_double, ctypes.c_int64,
                                ctypes.c_uint64]
        L.orc_relax.restype = ctypes.c_int64
        L.orc_max_torque.argtypes = [ctypes.POINTER(_System), P]
        L.orc_max_torque.restype = ctypes.c_double
        L.orc_llg_rhs.argtypes = [ctypes.c_double, ctypes.c_double, P, P, P]
        L.orc_neighbours.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, P, P, P, P, P, ctypes.c_int64]
        L.orc_neighbours.restype = ctypes.c_int64
        L.orc_greedy_colours.argtypes = [ctypes.c_int64, P, P, P]
        L.orc_greedy_colours.restype = ctypes.c_int
        L.orc_greedy_colours_in.argtypes = [ctypes.c_int64, P, P, P, P]
        L.orc_greedy_colours_in.restype = ctypes.c_int
        L.orc_lattice_visit.argtypes = [ctypes.c_int64, ctypes.c_int, P, P]
        L.orc_lattice_visit.restype = ctypes.c_int
        L.orc_mc_cone_width.argtypes = [ctypes.c_double]
        L.orc_mc_cone_width.restype = ctypes.c_double
        L.orc_mc_choice.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, P, P]
        L.orc_mc_run.argtypes = [ctypes.POINTER(_System), P, ctypes.c_uint64, ctypes.c_int64, P, P, P]
        L.orc_mc_run.restype = ctypes.c_int
        L.orc_mc_run_visit.argtypes = [ctypes.POINTER(_System), P, P, ctypes.c_uint64, ctypes.c_int64, P, P, P]
        L.orc_mc_run_visit.restype = ctypes.c_int
        L.orc_mc_run_random.argtypes = [ctypes.POINTER(_System), P, ctypes.c_uint64, ctypes.c_int64, P, P, P]
        L.orc_mc_run_random.restype = ctypes.c_int
        L.orc_demag_update.argtypes = [ctypes.POINTER(_System), P]
        L.orc_demag_update.restype = ctypes.c_int
        L.orc_demag_sample.argtypes = [ctypes.POINTER(_System), P, ctypes.c_int64, P, P]
        L.orc_demag_sample.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays: ctr uint32 [m, 4], key uint32 [m, 2] -> uint32 [m, 4]."""
    ctr = np.ascontiguousarray(np.atleast_2d(ctr), dtype=np.uint32)
    key = np.ascontiguousarray(np.atleast_2d(key), dtype=np.uint32)
    if key.shape[0] == 1 and ctr.shape[0] > 1:
        key = np.ascontiguousarray(np.repeat(key, ctr.shape[0], axis=0))
    out = np.empty_like(ctr)
    lib().orc_philox_batch(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def gaussians(seed, step, sites, purpose=0):
    """Thermal normals Gamma (shape [m, 3]) for the given sites at one step."""
    sites = np.ascontiguousarray(sites, dtype=np.uint64)
    out = np.empty((sites.size, 3), dtype=np.float64)
    lib().orc_gaussian3_batch(int(seed), int(step), sites.size, _ptr(sites), int(purpose), _ptr(out))
    return out


def greedy_colours(row_ptr, col):
    """Colour of every site: the smallest colour no neighbour with a lower
    index has.  Returns (colours int32 [n], number of colours)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = row_ptr.size - 1
    colour = np.zeros(max(n, 1), dtype=np.int32)
    k = lib().orc_greedy_colours(n, _ptr(row_ptr), _ptr(col), _ptr(colour))
    if k < 0:
        raise MemoryError("oracle colouring failed")
    return colour[:n], int(k)


def mc_cone_width(temperature):
    """Width of the Gaussian trial move, (2/25)(kB T/muB)^(1/5)."""
    return float(lib().orc_mc_cone_width(float(temperature)))


def mc_choice(seed, step, site):
    """Move type (0 flip, 1 Gaussian, 2 random) and acceptance uniform."""
    move = ctypes.c_uint32()
    u = ctypes.c_double()
    lib().orc_mc_choice(int(seed), int(step), int(site), ctypes.byref(move), ctypes.byref(u))
    return int(move.value), float(u.value)


def llg_rhs(gamma, alpha, spin, h):
    spin = np.ascontiguousarray(spin, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.empty(3)
    lib().orc_llg_rhs(float(gamma), float(alpha), _ptr(spin), _ptr(h), _ptr(out))
    return out


def neighbours(pos, box, shells, max_degree=64):
    """Brute-force neighbour list.  box: 3 lengths (0 = open axis);
    shells: list of (r_lo, r_hi), one per interaction type."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    box = np.ascontiguousarray(box, dtype=np.float64)
    lo = np.ascontiguousarray([s[0] for s in shells], dtype=np.float64)
    hi = np.ascontiguousarray([s[1] for s in shells], dtype=np.float64)
    cap = n * max_degree
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(cap, dtype=np.int32)
    ntype = np.zeros(cap, dtype=np.uint8)
    cnt = lib().orc_neighbours(n, _ptr(pos), _ptr(box), len(shells), _ptr(lo), _ptr(hi),
                               _ptr(row_ptr), _ptr(col), _ptr(ntype), cap)
    if cnt < 0:
        raise RuntimeError("neighbour capacity exceeded")
    return row_ptr, col[:cnt].copy(), ntype[:cnt].copy()


class System:
    """A spin system held in the arrays the C oracle reads.

    Construct from a ``spin_systems.Workload`` (or anything with the same
    attributes).  Temperature and applied field can be changed between
    calls, which is how the sweep protocols continue from one point to the
    next.
    """

    def __init__(self, w):
        lat = w.lattice
        self.n = lat.n
        self.dims = None if getattr(lat, "dims", None) is None else tuple(int(d) for d in lat.dims)
        self.row_ptr = np.ascontiguousarray(lat.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(lat.col, dtype=np.int32)
        self.ntype = np.ascontiguousarray(lat.ntype, dtype=np.uint8)
        self.J = np.ascontiguousarray(w.J, dtype=np.float64)
        self.mu_s = np.ascontiguousarray(np.broadcast_to(w.mu_s, (self.n,)), dtype=np.float64)
        self.k_u = np.ascontiguousarray(np.broadcast_to(w.k_u, (self.n,)), dtype=np.float64)
        self.easy_axis = np.ascontiguousarray(np.broadcast_to(w.easy_axis, (self.n, 3)),
                                              dtype=np.float64)
        self.alpha, self.gamma, self.dt = float(w.alpha), float(w.gamma), float(w.dt)
        self.temperature = float(w.temperature)
        self.H = np.array(w.H, dtype=np.float64)
        self.seed = int(w.seed)
        Jt = getattr(w, "J_tensor", None)
        self.J_tensor = None if Jt is None else np.ascontiguousarray(Jt, dtype=np.float64).reshape(-1, 9)
        kc = getattr(w, "k_c", None)
        self.k_c = None if kc is None else np.ascontiguousarray(np.broadcast_to(kc, (self.n,)),
                                                                dtype=np.float64)
        dm = getattr(w, "demag", None)
        self._demag = None
        if dm is not None:
            # the field and its valid flag persist across calls, like the library's
            self._demag_pos = np.ascontiguousarray(dm["pos"], dtype=np.float64).reshape(self.n, 3)
            self._demag_field = np.zeros((self.n, 3))
            self._demag = _Demag(self._demag_pos.ctypes.data, float(dm["cell_size"]),
                                 float(dm["atom_volume"]), int(dm["every"]), self._demag_field.ctypes.data,
                                 0, 0)

    def _struct(self):
        s = _System()
        s.n = self.n
        s.row_ptr = self.row_ptr.ctypes.data
        s.col = self.col.ctypes.data if self.col.size else None
        s.ntype = self.ntype.ctypes.data if self.ntype.size else None
        s.J = self.J.ctypes.data
        s.n_types = self.J.size
        s.mu_s = self.mu_s.ctypes.data
        s.k_u = self.k_u.ctypes.data
        s.easy_axis = self.easy_axis.ctypes.data
        s.alpha, s.gamma, s.dt = self.alpha, self.gamma, self.dt
        s.temperature = self.temperature
        s.H = (ctypes.c_double * 3)(*[float(v) for v in self.H])
        s.seed = self.seed
        s.J_tensor = None if self.J_tensor is None else self.J_tensor.ctypes.data
        s.k_c = None if self.k_c is None else self.k_c.ctypes.data
        s.demag = ctypes.pointer(self._demag) if self._demag is not None else None
        return s

    def demag_field(self, S):
        """Recompute the macrocell demagnetising field from S and return it
        per atom ([n, 3] tesla) with the number of macrocells."""
        st = self._struct()
        rc = lib().orc_demag_update(ctypes.byref(st), _ptr(np.ascontiguousarray(S, dtype=np.float64)))
        if rc != 0:
            raise MemoryError("oracle demagnetising field failed")
        return self._demag_field.copy(), int(self._demag.n_cells)

    def demag_sample(self, S, sites):
        """The demagnetising field computed from S at the given sites only
        ([len(sites), 3] tesla); the held field is left as it was."""
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.empty((sites.size, 3))
        st = self._struct()
        rc = lib().orc_demag_sample(ctypes.byref(st), _ptr(np.ascontiguousarray(S, dtype=np.float64)),
                                    int(sites.size), _ptr(sites), _ptr(out))
        if rc != 0:
            raise ValueError(f"oracle demagnetising sample failed ({rc})")
        return out

    def integrate(self, S, step0, n_steps, record=True):
        """Heun steps step0 .. step0+n_steps-1 in place on S ([n, 3] float64).
        Returns (m [n_steps, 3], E [n_steps]) when record, else (None, None)."""
        assert S.dtype == np.float64 and S.flags.c_contiguous and S.shape == (self.n, 3)
        m = np.empty((n_steps, 3)) if record else None
        E = np.empty(n_steps) if record else None
        st = self._struct()
        rc = lib().orc_integrate(ctypes.byref(st), _ptr(S), int(step0), int(n_steps),
                                 _ptr(m) if record else None, _ptr(E) if record else None)
        if rc != 0:
            raise FloatingPointError(f"oracle integrate failed ({rc})")
        return m, E

    def lattice_visit(self):
        """The colouring's visiting order grouped by basis site and cell
        parity (orc_lattice_visit) of the workload's cell grid."""
        if self.dims is None:
            raise ValueError("the workload has no cell grid")
        cells = np.asarray(self.dims, dtype=np.int32)
        nb = self.n // int(np.prod(cells))
        visit = np.empty(self.n, dtype=np.int64)
        if lib().orc_lattice_visit(self.n, nb, _ptr(cells), _ptr(visit)) != 0:
            raise ValueError("cell grid does not match the number of sites")
        return visit

    def colours(self, visit=None):
        """Greedy colour of every site (visit: the visiting order, None for
        ascending sites, "lattice" for lattice_visit())."""
        if isinstance(visit, str):
            visit = self.lattice_visit()
        colour = np.empty(self.n, dtype=np.int32)
        v = None if visit is None else np.ascontiguousarray(visit, dtype=np.int64)
        nc = lib().orc_greedy_colours_in(self.n, _ptr(self.row_ptr), _ptr(self.col), None if v is None else _ptr(v),
                                         _ptr(colour))
        if nc < 0:
            raise MemoryError("oracle colouring failed")
        return colour

    def mc(self, S, step0, n_steps, record=True, order="colour", visit=None):
        """Monte Carlo steps step0 .. step0+n_steps-1 (Hinzke-Nowak moves)
        in place on S; order "colour" (colour-class sweeps, every site once)
        or "random" (the paper's: N trials on random sites).  visit: the
        colouring's visiting order (None: ascending sites; "lattice":
        grouped by basis site and cell parity).  Returns (m [n_steps, 3],
        E [n_steps], accepted trials [n_steps]); m and E are None unless
        record."""
        assert S.dtype == np.float64 and S.flags.c_contiguous and S.shape == (self.n, 3)
        assert order in ("colour", "random")
        m = np.empty((n_steps, 3)) if record else None
        E = np.empty(n_steps) if record else None
        acc = np.empty(n_steps, dtype=np.int64)
        st = self._struct()
        outs = (_ptr(m) if record else None, _ptr(E) if record else None, _ptr(acc))
        if order == "random":
            rc = lib().orc_mc_run_random(ctypes.byref(st), _ptr(S), int(step0), int(n_steps), *outs)
        else:
            if isinstance(visit, str):
                visit = self.lattice_visit()
            v = None if visit is None else np.ascontiguousarray(visit, dtype=np.int64)
            rc = lib().orc_mc_run_visit(ctypes.byref(st), None if v is None else _ptr(v), _ptr(S), int(step0),
                                        int(n_steps), *outs)
        if rc != 0:
            raise MemoryError(f"oracle Monte Carlo failed ({rc})")
        return m, E, acc

    def energy(self, S):
        st = self._struct()
        return lib().orc_energy(ctypes.byref(st), _ptr(np.ascontiguousarray(S, dtype=np.float64)))

    def magnetisation(self, S):
        st = self._struct()
        out = np.empty(3)
        lib().orc_magnetisation(ctypes.byref(st), _ptr(np.ascontiguousarray(S, dtype=np.float64)),
                                _ptr(out))
        return out

    def fields(self, S):
        """Deterministic effective field (exchange + anisotropy + applied), [n, 3] tesla."""
        st = self._struct()
        out = np.empty((self.n, 3))
        lib().orc_effective_fields(ctypes.byref(st), _ptr(np.ascontiguousarray(S, dtype=np.float64)),
                                   _ptr(out))
        return out

    def max_torque(self, S):
        st = self._struct()
        return lib().orc_max_torque(ctypes.byref(st), _ptr(np.ascontiguousarray(S, dtype=np.float64)))

    def relax(self, S, torque_tol=1e-6, max_steps=10_000_000, step0=0):
        st = self._struct()
        return int(lib().orc_relax(ctypes.byref(st), _ptr(S), float(torque_tol), int(max_steps),
                                   int(step0)))


def block_stats(x, n_blocks):
    """Mean of a series and its standard error from n_blocks equal blocks
    (the series is cut to a multiple of n_blocks)."""
    x = np.asarray(x, dtype=np.float64)
    b = x.size // n_blocks
    if b == 0:
        return float(x.mean()), float("nan")
    means = x[: b * n_blocks].reshape(n_blocks, b).mean(axis=1)
    return float(x.mean()), float(means.std(ddof=1) / np.sqrt(n_blocks))


def average(sys: System, S, step0, n_eq, n_avg, n_blocks=10):
    """Equilibrate n_eq steps, then average over n_avg steps sampled after
    every step.  Returns (dict, next_step).  The dict holds <|m|> and its
    blocked standard error, <m> (3), <E> and its standard error."""
    sys.integrate(S, step0, n_eq, record=False)
    m, E = sys.integrate(S, step0 + n_eq, n_avg, record=True)
    mabs = np.sqrt((m * m).sum(axis=1))
    mean_abs, se_abs = block_stats(mabs, n_blocks)
    mean_E, se_E = block_stats(E, n_blocks)
    out = {"m_abs": mean_abs, "m_abs_se": se_abs, "m": m.mean(axis=0), "E": mean_E,
           "E_se": se_E}
    return out, step0 + n_eq + n_avg


def mc_average(sys: System, S, step0, n_eq, n_avg, n_blocks=10, order="colour", visit=None):
    """Monte Carlo counterpart of average(): n_eq steps to equilibrate, then
    n_avg steps sampled after every step (trial order as in System.mc)."""
    sys.mc(S, step0, n_eq, record=False, order=order, visit=visit)
    m, E, acc = sys.mc(S, step0 + n_eq, n_avg, record=True, order=order, visit=visit)
    mabs = np.sqrt((m * m).sum(axis=1))
    mean_abs, se_abs = block_stats(mabs, n_blocks)
    mean_E, se_E = block_stats(E, n_blocks)
    out = {"m_abs": mean_abs, "m_abs_se": se_abs, "m": m.mean(axis=0), "E": mean_E,
           "E_se": se_E, "acceptance": float(acc.sum()) / (sys.n * n_avg)}
    return out, step0 + n_eq + n_avg


def sweep_temperature(sys: System, S, temperatures, n_eq, n_avg, step0=0, n_blocks=10):
    """Heating ramp with continuation: the final state at one temperature is
    the starting state at the next; the step counter keeps running."""
    rows = []
    step = step0
    for T in temperatures:
        sys.temperature = float(T)
        r, step = average(sys, S, step, n_eq, n_avg, n_blocks)
        r["T"] = float(T)
        rows.append(r)
    return rows, step


def sweep_field(sys: System, S, fields, n_eq, n_avg, step0=0, n_blocks=10):
    """Field sweep with continuation; each entry of fields is a 3-vector."""
    rows = []
    step = step0
    for H in fields:
        sys.H = np.asarray(H, dtype=np.float64)
        r, step = average(sys, S, step, n_eq, n_avg, n_blocks)
        r["H"] = np.asarray(H, dtype=np.float64)
        rows.append(r)
    return rows, step
