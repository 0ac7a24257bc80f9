"""Python binding of libsllg (stochastic LLG + Heun on MI355X).

Argument marshalling only: every step of the dynamics runs in the HIP
kernels of ``libsllg.so``; this module converts numpy arrays (and torch
tensors / streams, when given) into the C ABI declared in
``include/sllg.h``.  If the library is not built the import of any entry
point raises at once; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsllg.so")

FP32, FP64 = 0, 1
STATUS = {0: "SLLG_OK", -1: "SLLG_E_ARG", -2: "SLLG_E_NOMEM", -3: "SLLG_E_DEVICE",
          -4: "SLLG_E_STATE", -5: "SLLG_E_BUDGET", -6: "SLLG_E_NUMERIC", -7: "SLLG_E_CANCELLED"}

# every symbol include/sllg.h declares
EXPORTS = [
    "sllg_create", "sllg_destroy", "sllg_last_error", "sllg_status_string", "sllg_set_neighbours",
    "sllg_set_lattice",
    "sllg_set_materials", "sllg_set_exchange_tensors", "sllg_set_cubic_anisotropy", "sllg_set_demag",
    "sllg_demag_field", "sllg_set_integrator", "sllg_set_conditions", "sllg_set_rng",
    "sllg_get_step", "sllg_set_spins", "sllg_get_spins", "sllg_integrate", "sllg_integrate_dev",
    "sllg_measure", "sllg_average", "sllg_sweep_temperature", "sllg_sweep_field",
    "sllg_max_torque", "sllg_relax", "sllg_hysteresis", "sllg_thermal_normals", "sllg_thermal_normals_noalloc", "sllg_autotune", "sllg_mc", "sllg_mc_average", "sllg_checkpoint_size", "sllg_checkpoint", "sllg_restore",
    "sllg_set_option", "sllg_get_option",
    "sllg_server_create", "sllg_server_destroy", "sllg_server_last_error", "sllg_submit",
    "sllg_poll", "sllg_wait", "sllg_fetch", "sllg_cancel", "sllg_release", "sllg_server_get_stats",
    "sllg_server_clock", "sllg_build_sc", "sllg_build_bcc", "sllg_build_fcc_sphere",
]


class SllgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


_lib = None
P = ctypes.c_void_p
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
D = ctypes.c_double


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_int),
                ("chunk_steps", ctypes.c_int), ("precision", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("n_spins", I64), ("row_ptr", P), ("col", P), ("ntype", P), ("J", P),
                ("n_types", ctypes.c_int), ("mu_s", P), ("k_u", P), ("easy_axis", P),
                ("per_site", ctypes.c_int), ("S0", P), ("alpha", D), ("gamma", D), ("dt", D),
                ("temperature", D), ("H_app", D * 3), ("seed", U64), ("n_steps", I64),
                ("n_avg", I64), ("record", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("n_spins", I64), ("n_steps", I64),
                ("steps_done", I64), ("m", D * 3), ("E", D), ("avg", D * 8), ("t_submit", D),
                ("t_start", D), ("t_done", D), ("hbm_bytes", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", I64), ("completed", I64), ("failed", I64), ("cancelled", I64),
                ("active", I64), ("queued", I64), ("hbm_in_use", ctypes.c_size_t),
                ("hbm_budget", ctypes.c_size_t), ("spin_steps", D), ("busy_seconds", D),
                ("chunks", I64), ("tuned_compositions", I64), ("last_xcd_remap", I64),
                ("last_tile_order", I64)]


def lib():
    """Load libsllg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    c = ctypes.c_int
    sig = {
        "sllg_create": (c, [c, c, I64, ctypes.POINTER(P)]),
        "sllg_destroy": (None, [P]),
        "sllg_last_error": (ctypes.c_char_p, [P]),
        "sllg_status_string": (ctypes.c_char_p, [c]),
        "sllg_set_neighbours": (c, [P, P, P, P, P, c]),
        "sllg_set_lattice": (c, [P, c, P, P]),
        "sllg_set_materials": (c, [P, P, P, P, c]),
        "sllg_set_exchange_tensors": (c, [P, P, c]),
        "sllg_max_torque": (c, [P, P, P]),
        "sllg_set_demag": (c, [P, P, D, D, I64]),
        "sllg_demag_field": (c, [P, P, P]),
        "sllg_relax": (c, [P, D, I64, I64, P, P, P]),
        "sllg_hysteresis": (c, [P, P, I64, D, I64, I64, P, P, P]),
        "sllg_set_cubic_anisotropy": (c, [P, P, c]),
        "sllg_set_integrator": (c, [P, D, D, D]),
        "sllg_set_conditions": (c, [P, D, P]),
        "sllg_set_rng": (c, [P, U64, U64]),
        "sllg_get_step": (c, [P, ctypes.POINTER(U64)]),
        "sllg_set_spins": (c, [P, P]),
        "sllg_get_spins": (c, [P, P]),
        "sllg_integrate": (c, [P, I64, P, P, P]),
        "sllg_integrate_dev": (c, [P, I64, P, P, P]),
        "sllg_measure": (c, [P, P, P, P]),
        "sllg_average": (c, [P, I64, I64, c, P, P]),
        "sllg_sweep_temperature": (c, [P, P, I64, I64, I64, c, P, P]),
        "sllg_sweep_field": (c, [P, P, I64, I64, I64, c, P, P]),
        "sllg_thermal_normals": (c, [c, c, U64, U64, I64, P]),
        "sllg_thermal_normals_noalloc": (c, [c, c, U64, U64, I64, P]),
        "sllg_autotune": (c, [P, c, ctypes.POINTER(D), P]),
        "sllg_mc": (c, [P, I64, P, P, P, P]),
        "sllg_mc_average": (c, [P, I64, I64, c, P, P]),
        "sllg_checkpoint_size": (c, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "sllg_checkpoint": (c, [P, P, ctypes.c_size_t]),
        "sllg_restore": (c, [P, P, ctypes.c_size_t]),
        "sllg_set_option": (c, [P, ctypes.c_char_p, I64]),
        "sllg_get_option": (c, [P, ctypes.c_char_p, ctypes.POINTER(I64)]),
        "sllg_server_create": (c, [c, ctypes.POINTER(ServerOpts), ctypes.POINTER(P)]),
        "sllg_server_destroy": (None, [P]),
        "sllg_server_last_error": (ctypes.c_char_p, [P]),
        "sllg_submit": (c, [P, ctypes.POINTER(Request), ctypes.POINTER(U64)]),
        "sllg_poll": (c, [P, U64, ctypes.POINTER(Result)]),
        "sllg_wait": (c, [P, U64, D, ctypes.POINTER(Result)]),
        "sllg_fetch": (c, [P, U64, P, P, P]),
        "sllg_cancel": (c, [P, U64]),
        "sllg_release": (c, [P, U64]),
        "sllg_server_get_stats": (c, [P, ctypes.POINTER(ServerStats)]),
        "sllg_server_clock": (D, [P]),
        "sllg_build_sc": (c, [P, P, ctypes.POINTER(I64), ctypes.POINTER(I64), P, P, P, P]),
        "sllg_build_bcc": (c, [P, P, c, ctypes.POINTER(I64), ctypes.POINTER(I64), P, P, P, P]),
        "sllg_build_fcc_sphere": (c, [D, D, ctypes.POINTER(I64), ctypes.POINTER(I64), P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(P)


def _dev_ptr(x):
    """Device pointer of a torch tensor (or an int address)."""
    if x is None:
        return None
    if isinstance(x, int):
        return P(x)
    return P(x.data_ptr())


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return P(stream)
    return P(stream.cuda_stream)


def _c64(a, dtype=np.float64, shape=None):
    a = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None:
        a = a.reshape(shape)
    return a


def thermal_normals(seed, step, n, precision=FP64, device=0):
    """Gamma [n, 3] of sites 0..n-1 at one step, as the kernels draw them."""
    out = np.empty((n, 3), dtype=np.float64)
    st = lib().sllg_thermal_normals(device, precision, int(seed), int(step), int(n), _ptr(out))
    if st != 0:
        raise SllgError(st, "thermal_normals failed")
    return out


def thermal_normals_noalloc(seed, step, n, precision=FP64, device=0):
    """thermal_normals through the entry point that allocates no device
    memory (sllg_thermal_normals_noalloc; n <= 2^18)."""
    out = np.empty((n, 3), dtype=np.float64)
    st = lib().sllg_thermal_normals_noalloc(device, precision, int(seed), int(step), int(n), _ptr(out))
    if st != 0:
        raise SllgError(st, lib().sllg_last_error(None).decode())
    return out


def _built(call):
    """Run a structure builder of the C ABI twice (counts, then the arrays):
    (row_ptr int64 [n + 1], col int32 [nnz], type uint8 [nnz], pos [n, 3])."""
    n, nnz = I64(0), I64(0)
    st = call(ctypes.byref(n), ctypes.byref(nnz), None, None, None, None)
    if st != 0:
        raise SllgError(st, lib().sllg_last_error(None).decode())
    row_ptr = np.empty(n.value + 1, dtype=np.int64)
    col = np.empty(max(nnz.value, 1), dtype=np.int32)
    typ = np.empty(max(nnz.value, 1), dtype=np.uint8)
    pos = np.empty((n.value, 3), dtype=np.float64)
    st = call(ctypes.byref(n), ctypes.byref(nnz), _ptr(row_ptr), _ptr(col), _ptr(typ), _ptr(pos))
    if st != 0:
        raise SllgError(st, lib().sllg_last_error(None).decode())
    return row_ptr, col[:nnz.value], typ[:nnz.value], pos


def build_sc(cells, periodic=(1, 1, 1)):
    """Simple-cubic CSR neighbour list from the C ABI (sllg_build_sc)."""
    c = np.ascontiguousarray(cells, dtype=np.int32).reshape(3)
    p = np.ascontiguousarray(periodic, dtype=np.int32).reshape(3)
    return _built(lambda n, nnz, rp, col, ty, pos: lib().sllg_build_sc(_ptr(c), _ptr(p), n, nnz, rp, col, ty, pos))


def build_bcc(cells, periodic=(1, 1, 1), second_neighbours=False):
    """bcc CSR neighbour list from the C ABI (sllg_build_bcc)."""
    c = np.ascontiguousarray(cells, dtype=np.int32).reshape(3)
    p = np.ascontiguousarray(periodic, dtype=np.int32).reshape(3)
    return _built(lambda n, nnz, rp, col, ty, pos: lib().sllg_build_bcc(_ptr(c), _ptr(p), int(bool(second_neighbours)),
                                                                        n, nnz, rp, col, ty, pos))


def build_fcc_sphere(a_nm, radius_nm):
    """fcc sphere CSR neighbour list from the C ABI (sllg_build_fcc_sphere)."""
    return _built(lambda n, nnz, rp, col, ty, pos: lib().sllg_build_fcc_sphere(float(a_nm), float(radius_nm), n, nnz,
                                                                               rp, col, ty, pos))


class SpinSystem:
    """One spin system on the GPU (a handle of the C ABI)."""

    def __init__(self, n, precision=FP32, device=0):
        self._h = P()
        L = lib()
        st = L.sllg_create(int(device), int(precision), int(n), ctypes.byref(self._h))
        if st != 0:
            raise SllgError(st, L.sllg_last_error(None).decode())
        self.n = int(n)
        self.precision = precision

    def close(self):
        if self._h:
            lib().sllg_destroy(self._h)
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != 0:
            raise SllgError(st, lib().sllg_last_error(self._h).decode())

    # ---- set-up ----------------------------------------------------------
    def set_neighbours(self, row_ptr, col, ntype, J):
        row_ptr = _c64(row_ptr, np.int64)
        col = _c64(col, np.int32)
        ntype = None if ntype is None else _c64(ntype, np.uint8)
        J = _c64(np.atleast_1d(J))
        self._check(lib().sllg_set_neighbours(self._h, _ptr(row_ptr), _ptr(col), _ptr(ntype), _ptr(J),
                                              int(J.size)))

    def set_lattice(self, n_basis, cells, periodic):
        """Declare site i = b + n_basis (x + cells[0] (y + cells[1] z))
        (sllg_set_lattice): lets the library take the fused step."""
        cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(3)
        per = np.ascontiguousarray([1 if p else 0 for p in periodic], dtype=np.int32).reshape(3)
        self._check(lib().sllg_set_lattice(self._h, int(n_basis), _ptr(cells), _ptr(per)))

    def set_materials(self, mu_s, k_u, easy_axis, per_site=None):
        mu_s = _c64(np.atleast_1d(mu_s))
        k_u = _c64(np.atleast_1d(k_u))
        axis = _c64(easy_axis).reshape(-1)
        if per_site is None:
            per_site = 1 if mu_s.size > 1 else 0
        self._check(lib().sllg_set_materials(self._h, _ptr(mu_s), _ptr(k_u), _ptr(axis), int(per_site)))

    def set_exchange_tensors(self, J):
        """Exchange tensors [n_types, 3, 3] (joules per link) for the
        neighbour list's types; None returns to the scalar table."""
        if J is None:
            self._check(lib().sllg_set_exchange_tensors(self._h, None, 0))
            return
        J = _c64(J).reshape(-1, 9)
        self._check(lib().sllg_set_exchange_tensors(self._h, _ptr(J), int(J.shape[0])))

    def set_cubic_anisotropy(self, k_c, per_site=None):
        """Cubic anisotropy constants k_c (J/atom): one value or one per
        site; None removes it."""
        if k_c is None:
            self._check(lib().sllg_set_cubic_anisotropy(self._h, None, 0))
            return
        k_c = _c64(np.atleast_1d(k_c))
        if per_site is None:
            per_site = 1 if k_c.size > 1 else 0
        self._check(lib().sllg_set_cubic_anisotropy(self._h, _ptr(k_c), int(per_site)))

    def set_integrator(self, alpha, gamma, dt):
        self._check(lib().sllg_set_integrator(self._h, float(alpha), float(gamma), float(dt)))

    def set_conditions(self, temperature, H=(0.0, 0.0, 0.0)):
        H = _c64(H)
        self._check(lib().sllg_set_conditions(self._h, float(temperature), _ptr(H)))

    def set_rng(self, seed, step=0):
        self._check(lib().sllg_set_rng(self._h, int(seed), int(step)))

    @property
    def step(self):
        v = U64()
        self._check(lib().sllg_get_step(self._h, ctypes.byref(v)))
        return int(v.value)

    def set_spins(self, S):
        S = _c64(S).reshape(-1)
        self._check(lib().sllg_set_spins(self._h, _ptr(S)))

    def get_spins(self):
        out = np.empty((self.n, 3))
        self._check(lib().sllg_get_spins(self._h, _ptr(out)))
        return out

    def set_option(self, key, value):
        self._check(lib().sllg_set_option(self._h, key.encode(), int(value)))

    def get_option(self, key):
        v = I64()
        self._check(lib().sllg_get_option(self._h, key.encode(), ctypes.byref(v)))
        return int(v.value)

    # ---- dynamics --------------------------------------------------------
    def integrate(self, n_steps, record=True, stream=None):
        """Advance n_steps; returns (m [n,3], E [n]) when record else (None, None)."""
        m = np.empty((n_steps, 3)) if record else None
        E = np.empty(n_steps) if record else None
        self._check(lib().sllg_integrate(self._h, int(n_steps), _ptr(m), _ptr(E), _stream(stream)))
        return m, E

    def integrate_dev(self, n_steps, m_dev=None, E_dev=None, stream=None):
        """Advance n_steps with m/E written to device tensors (torch) or raw
        addresses; asynchronous on `stream` (a torch stream or address)."""
        self._check(lib().sllg_integrate_dev(self._h, int(n_steps), _dev_ptr(m_dev), _dev_ptr(E_dev),
                                             _stream(stream)))

    def autotune(self, trial_steps=20, stream=None):
        """Pick the fastest launch shape for this system (state unchanged);
        returns (us per step, chosen options)."""
        us = D()
        self._check(lib().sllg_autotune(self._h, int(trial_steps), ctypes.byref(us), _stream(stream)))
        keys = ["graph_steps"]
        if self.get_option("fused_active"):
            keys += ["fused_tile_x", "fused_tile_y", "fused_planes", "fused_threads"]
        else:
            keys += ["tile_sites", "xcd_remap", "grid_scale_pct", "tile_order", "lds_window"]
        return us.value, {k: self.get_option(k) for k in keys}

    def set_demag(self, pos, cell_size, atom_volume, every):
        """Macrocell demagnetising field: atom positions [n, 3] (m), cell
        edge (m), atomic volume (m^3), update interval (steps); pos None
        switches it off."""
        if pos is None:
            self._check(lib().sllg_set_demag(self._h, None, 0.0, 0.0, 1))
            return
        pos = _c64(pos).reshape(-1)
        self._check(lib().sllg_set_demag(self._h, _ptr(pos), float(cell_size), float(atom_volume), int(every)))

    def demag_field(self, stream=None):
        """The demagnetising field in effect, per atom [n, 3] tesla: the
        field held since the last scheduled update, or, when none is held
        yet, the field of the current spins (computed now and held)."""
        out = np.empty((self.n, 3))
        self._check(lib().sllg_demag_field(self._h, _ptr(out), _stream(stream)))
        return out

    def max_torque(self, stream=None):
        """Largest |S_i x H_i| (tesla) of the current state."""
        t = D()
        self._check(lib().sllg_max_torque(self._h, ctypes.byref(t), _stream(stream)))
        return t.value

    def relax(self, torque_tol=1e-6, max_steps=10_000_000, check_every=1, stream=None):
        """Heun steps at T = 0 until the largest torque is at most
        torque_tol.  Returns (steps taken, final torque); raises SllgError
        (SLLG_E_NUMERIC) when max_steps do not suffice."""
        n = ctypes.c_int64()
        t = D()
        self._check(lib().sllg_relax(self._h, float(torque_tol), int(max_steps), int(check_every),
                                     ctypes.byref(n), ctypes.byref(t), _stream(stream)))
        return n.value, t.value

    def hysteresis(self, H, torque_tol=1e-6, max_steps=10_000_000, check_every=1, stream=None):
        """Quasi-static loop over the fields H [n, 3]: relax at each, record
        the reduced magnetisation.  Returns (m [n, 3], steps [n]; -1 where
        max_steps did not suffice)."""
        H = _c64(H).reshape(-1, 3)
        m = np.empty((H.shape[0], 3))
        steps = np.empty(H.shape[0], dtype=np.int64)
        self._check(lib().sllg_hysteresis(self._h, _ptr(H), H.shape[0], float(torque_tol), int(max_steps),
                                          int(check_every), _ptr(m), _ptr(steps), _stream(stream)))
        return m, steps

    def mc(self, n_steps, record=True, stream=None):
        """Monte Carlo steps (Hinzke-Nowak moves, colour-class sweeps).
        Returns (m [n, 3], E [n], accepted trials [n]); m and E are None
        unless record."""
        m = np.empty((n_steps, 3)) if record else None
        E = np.empty(n_steps) if record else None
        acc = np.empty(n_steps, dtype=np.int64)
        self._check(lib().sllg_mc(self._h, int(n_steps), _ptr(m), _ptr(E), _ptr(acc), _stream(stream)))
        return m, E, acc

    def mc_average(self, n_eq, n_avg, n_blocks=10, stream=None):
        """Monte Carlo thermal average (sllg_mc_average): n_eq steps, then
        n_avg steps sampled after every step.  Returns <|m|> and its blocked
        standard error, <m>, <E> and its standard error, and the acceptance
        rate."""
        out = np.empty(9)
        self._check(lib().sllg_mc_average(self._h, int(n_eq), int(n_avg), int(n_blocks), _ptr(out),
                                          _stream(stream)))
        return {"m_abs": out[0], "m_abs_se": out[1], "m": out[2:5].copy(), "E": out[5], "E_se": out[6],
                "acceptance": out[8]}

    def measure(self):
        m = np.empty(3)
        E = np.empty(1)
        self._check(lib().sllg_measure(self._h, _ptr(m), _ptr(E), None))
        return m, float(E[0])

    def average(self, n_eq, n_avg, n_blocks=10):
        out = np.empty(8)
        self._check(lib().sllg_average(self._h, int(n_eq), int(n_avg), int(n_blocks), _ptr(out), None))
        return _avg_dict(out)

    def sweep_temperature(self, temperatures, n_eq, n_avg, n_blocks=10):
        T = _c64(temperatures)
        out = np.empty((T.size, 8))
        self._check(lib().sllg_sweep_temperature(self._h, _ptr(T), T.size, int(n_eq), int(n_avg),
                                                 int(n_blocks), _ptr(out), None))
        return [_avg_dict(r) | {"T": float(t)} for r, t in zip(out, T)]

    def sweep_field(self, fields, n_eq, n_avg, n_blocks=10):
        H = _c64(fields).reshape(-1, 3)
        out = np.empty((H.shape[0], 8))
        self._check(lib().sllg_sweep_field(self._h, _ptr(np.ascontiguousarray(H)), H.shape[0], int(n_eq),
                                           int(n_avg), int(n_blocks), _ptr(out), None))
        return [_avg_dict(r) | {"H": h.copy()} for r, h in zip(out, H)]

    def checkpoint(self):
        size = ctypes.c_size_t()
        self._check(lib().sllg_checkpoint_size(self._h, ctypes.byref(size)))
        buf = np.empty(size.value, dtype=np.uint8)
        self._check(lib().sllg_checkpoint(self._h, _ptr(buf), size.value))
        return buf.tobytes()

    def restore(self, blob):
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        self._check(lib().sllg_restore(self._h, _ptr(buf), buf.size))


def _avg_dict(o):
    return {"m_abs": float(o[0]), "m_abs_se": float(o[1]), "m": np.array(o[2:5]), "E": float(o[5]),
            "E_se": float(o[6]), "n_blocks": int(o[7])}


def from_workload(w, precision=FP32, device=0, check_symmetry=True, stencil=1, lattice=True):
    """Build a SpinSystem from a spin_systems.Workload-like object.
    stencil=0 keeps the general SELL-64 neighbour layout; lattice=False
    leaves the cell grid of a crystal lattice undeclared (no fused step)."""
    s = SpinSystem(w.lattice.n, precision, device)
    if not check_symmetry:
        s.set_option("check_symmetry", 0)
    if not stencil:
        s.set_option("stencil", 0)
    lat = w.lattice
    s.set_neighbours(lat.row_ptr, lat.col, lat.ntype, w.J)
    if lattice and lat.dims is not None:
        cells = int(np.prod(lat.dims))
        if cells > 0 and lat.n % cells == 0:
            try:
                s.set_lattice(lat.n // cells, lat.dims, lat.periodic)
            except SllgError as err:
                # links beyond the next cell (long-range exchange): no cell
                # lattice in the library's sense
                if err.status != -1:   # SLLG_E_ARG
                    raise
    mu, ku, ax = np.asarray(w.mu_s), np.asarray(w.k_u), np.asarray(w.easy_axis)
    uniform = bool(np.all(mu == mu[0]) and np.all(ku == ku[0]) and np.all(ax == ax[0]))
    if uniform:
        s.set_materials(mu[:1], ku[:1], ax[:1], per_site=0)
    else:
        s.set_materials(mu, ku, ax, per_site=1)
    if getattr(w, "J_tensor", None) is not None:
        s.set_exchange_tensors(w.J_tensor)
    kc = getattr(w, "k_c", None)
    if kc is not None:
        kc = np.asarray(kc, dtype=np.float64)
        s.set_cubic_anisotropy(kc[:1] if np.all(kc == kc.flat[0]) else kc)
    dm = getattr(w, "demag", None)
    if dm is not None:
        s.set_demag(dm["pos"], dm["cell_size"], dm["atom_volume"], dm["every"])
    s.set_integrator(w.alpha, w.gamma, w.dt)
    s.set_conditions(w.temperature, w.H)
    s.set_rng(w.seed, 0)
    s.set_spins(w.S0)
    return s


REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


def _result_dict(r):
    return {"state": REQ_STATES.get(r.state, r.state), "status": STATUS.get(r.status, r.status),
            "n_spins": r.n_spins, "n_steps": r.n_steps, "steps_done": r.steps_done,
            "m": np.array(r.m[:]), "E": r.E, "avg": _avg_dict(np.array(r.avg[:])),
            "t_submit": r.t_submit, "t_start": r.t_start, "t_done": r.t_done,
            "hbm_bytes": int(r.hbm_bytes)}


class Server:
    """Continuous-batching request server (sllg_server_* of the C ABI)."""

    def __init__(self, hbm_budget=4 << 30, max_active=256, chunk_steps=64, precision=FP32, device=0):
        self._h = P()
        opts = ServerOpts(int(hbm_budget), int(max_active), int(chunk_steps), int(precision))
        st = lib().sllg_server_create(int(device), ctypes.byref(opts), ctypes.byref(self._h))
        if st != 0:
            raise SllgError(st, "server create failed")
        self.precision = precision
        self._keep = {}

    def close(self):
        if self._h:
            lib().sllg_server_destroy(self._h)
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != 0:
            raise SllgError(st, lib().sllg_server_last_error(self._h).decode())

    def submit(self, w, n_steps=None, n_avg=0, record=False, S0=None):
        """Queue one request built from a spin_systems.Workload (initial
        spins: S0 if given, else the workload's own)."""
        if S0 is None:
            S0 = w.S0
        lat = w.lattice
        n = lat.n
        arrays = {
            "row_ptr": _c64(lat.row_ptr, np.int64), "col": _c64(lat.col, np.int32),
            "ntype": _c64(lat.ntype, np.uint8), "J": _c64(np.atleast_1d(w.J)),
        }
        mu, ku, ax = np.asarray(w.mu_s), np.asarray(w.k_u), np.asarray(w.easy_axis)
        uniform = bool(np.all(mu == mu[0]) and np.all(ku == ku[0]) and np.all(ax == ax[0]))
        if uniform:
            arrays.update(mu_s=_c64(mu[:1]), k_u=_c64(ku[:1]), easy_axis=_c64(ax[:1]).reshape(-1))
        else:
            arrays.update(mu_s=_c64(mu), k_u=_c64(ku), easy_axis=_c64(ax).reshape(-1))
        if S0 is not None:
            arrays["S0"] = _c64(S0).reshape(-1)
        req = Request()
        req.n_spins = n
        req.row_ptr, req.col, req.ntype, req.J = (arrays[k].ctypes.data for k in ("row_ptr", "col", "ntype", "J"))
        req.n_types = arrays["J"].size
        req.mu_s, req.k_u, req.easy_axis = (arrays[k].ctypes.data for k in ("mu_s", "k_u", "easy_axis"))
        req.per_site = 0 if uniform else 1
        req.S0 = arrays["S0"].ctypes.data if "S0" in arrays else None
        req.alpha, req.gamma, req.dt, req.temperature = float(w.alpha), float(w.gamma), float(w.dt), float(w.temperature)
        req.H_app = (D * 3)(*[float(v) for v in w.H])
        req.seed = int(w.seed)
        req.n_steps = int(w.n_steps if n_steps is None else n_steps)
        req.n_avg = int(n_avg)
        req.record = 1 if record else 0
        t = U64()
        self._check(lib().sllg_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (n, req.n_steps, bool(record))
        return int(t.value)

    def poll(self, ticket):
        r = Result()
        self._check(lib().sllg_poll(self._h, int(ticket), ctypes.byref(r)))
        return _result_dict(r)

    def wait(self, ticket, timeout=60.0):
        r = Result()
        st = lib().sllg_wait(self._h, int(ticket), float(timeout), ctypes.byref(r))
        if st != 0:
            raise SllgError(st, f"request {ticket} not finished within {timeout} s")
        return _result_dict(r)

    def fetch(self, ticket):
        """(final spins, m series or None, E series or None) of a finished request."""
        n, n_steps, record = self._keep[ticket]
        S = np.empty((n, 3))
        m = np.empty((n_steps, 3)) if record else None
        E = np.empty(n_steps) if record else None
        self._check(lib().sllg_fetch(self._h, int(ticket), _ptr(S), _ptr(m), _ptr(E)))
        return S, m, E

    def cancel(self, ticket):
        self._check(lib().sllg_cancel(self._h, int(ticket)))

    def release(self, ticket):
        self._check(lib().sllg_release(self._h, int(ticket)))
        self._keep.pop(ticket, None)

    def stats(self):
        s = ServerStats()
        self._check(lib().sllg_server_get_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in ServerStats._fields_}

    def clock(self):
        return float(lib().sllg_server_clock(self._h))
