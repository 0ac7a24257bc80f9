"""CPU-side checks of the C-ABI library: it loads, exports every function
include/sllg.h declares, and rejects malformed input on the host (no GPU
needed: set-up calls validate and copy before the device is opened)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1310_6143_amd as sl
from spin_systems import sc_reference

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sllg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sllg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = sl.lib()
    names = _declared()
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(sl.EXPORTS) == names


def _valid_system(n=27):
    w = sc_reference(L=3)
    s = sl.SpinSystem(w.n, sl.FP64)
    return w, s


def _status(fn):
    with pytest.raises(sl.SllgError) as e:
        fn()
    return e.value.name


def test_rejects_malformed_neighbour_lists():
    w, s = _valid_system()
    lat = w.lattice
    rp, col, t = lat.row_ptr.copy(), lat.col.copy(), lat.ntype.copy()
    bad = col.copy()
    bad[0] = 0                                    # self link in row 0
    assert _status(lambda: s.set_neighbours(rp, bad, t, w.J)) == "SLLG_E_ARG"
    bad = col.copy()
    bad[3] = w.n                                  # out of range
    assert _status(lambda: s.set_neighbours(rp, bad, t, w.J)) == "SLLG_E_ARG"
    bad_rp = rp.copy()
    bad_rp[5] = bad_rp[4] - 1                     # decreasing row pointer
    assert _status(lambda: s.set_neighbours(bad_rp, col, t, w.J)) == "SLLG_E_ARG"
    tt = t.copy()
    tt[0] = 1                                     # type out of range for one J
    assert _status(lambda: s.set_neighbours(rp, col, tt, w.J)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_neighbours(rp, col, tt, [1e-21, 2e-21])) == "SLLG_E_ARG"  # asymmetric types
    assert _status(lambda: s.set_neighbours(rp, col, t, [np.nan])) == "SLLG_E_ARG"
    s.set_option("check_symmetry", 0)
    s.set_neighbours(rp, col, tt, [1e-21, 2e-21])  # accepted once the check is off
    s.set_option("check_symmetry", 1)
    s.set_neighbours(rp, col, t, w.J)
    s.close()


def test_rejects_bad_materials_spins_and_parameters():
    w, s = _valid_system()
    assert _status(lambda: s.set_materials([-1.0], [0.0], [0, 0, 1.0], 0)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_materials([1e-23], [np.inf], [0, 0, 1.0], 0)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_materials([1e-23], [0.0], [0, 0, 0.0], 0)) == "SLLG_E_ARG"
    S = np.tile([0, 0, 1.0], (w.n, 1))
    S[4] = 0.0
    assert _status(lambda: s.set_spins(S)) == "SLLG_E_ARG"
    S[4] = [np.nan, 0, 1]
    assert _status(lambda: s.set_spins(S)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_integrator(-0.1, 1.76e11, 1e-16)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_integrator(0.1, 1.76e11, 0.0)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_conditions(-1.0, [0, 0, 0])) == "SLLG_E_ARG"
    assert _status(lambda: s.set_conditions(10.0, [0, np.nan, 0])) == "SLLG_E_ARG"
    assert _status(lambda: s.set_option("no_such_option", 1)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_option("graph_steps", 3)) == "SLLG_E_ARG"
    # integrating before the set-up is complete is a state error
    assert _status(lambda: s.integrate(1)) == "SLLG_E_STATE"
    s.close()


def test_spins_are_normalised_and_kept_on_host_before_first_run():
    w, s = _valid_system()
    S = np.tile([0.0, 3.0, 4.0], (w.n, 1))
    s.set_spins(S)
    out = s.get_spins()
    assert np.allclose(out, np.tile([0, 0.6, 0.8], (w.n, 1)), atol=1e-15)
    assert s.step == 0
    s.set_rng(7, 123)
    assert s.step == 123
    s.close()


def test_checkpoint_round_trip_on_host():
    w, s = _valid_system()
    S = np.random.default_rng(0).standard_normal((w.n, 3))
    s.set_spins(S)
    s.set_rng(99, 4242)
    blob = s.checkpoint()
    s2 = sl.SpinSystem(w.n, sl.FP64)
    s2.restore(blob)
    assert s2.step == 4242
    assert np.array_equal(s2.get_spins(), s.get_spins())
    s3 = sl.SpinSystem(w.n + 1, sl.FP64)
    assert _status(lambda: s3.restore(blob)) == "SLLG_E_ARG"
    assert _status(lambda: s2.restore(blob[:20])) == "SLLG_E_ARG"
    for x in (s, s2, s3):
        x.close()


def test_create_rejects_bad_arguments():
    L = sl.lib()
    h = ctypes.c_void_p()
    assert L.sllg_create(0, 0, 0, ctypes.byref(h)) == -1
    assert L.sllg_create(0, 5, 10, ctypes.byref(h)) == -1
    assert L.sllg_create(0, 0, 1 << 28, ctypes.byref(h)) == -1
    assert L.sllg_status_string(-5) == b"SLLG_E_BUDGET"


def test_exchange_tensors_and_cubic_anisotropy_validation():
    from spin_systems import with_tensor_exchange
    w = with_tensor_exchange(sc_reference(L=4), D=1e-21, dmi="bulk")
    s = sl.SpinSystem(w.n, sl.FP64)
    assert _status(lambda: s.set_exchange_tensors(w.J_tensor)) == "SLLG_E_STATE"     # no neighbours yet
    assert _status(lambda: s.set_cubic_anisotropy([1e-24])) == "SLLG_E_STATE"       # no materials yet
    lat = w.lattice
    s.set_neighbours(lat.row_ptr, lat.col, lat.ntype, w.J)     # 6 directed types, equal J
    s.set_exchange_tensors(w.J_tensor)
    assert _status(lambda: s.set_exchange_tensors(w.J_tensor[:5])) == "SLLG_E_ARG"  # count
    bad = w.J_tensor.copy()
    bad[2] = bad[2].T                        # no longer the transpose of its reverse type
    assert _status(lambda: s.set_exchange_tensors(bad)) == "SLLG_E_ARG"
    bad = w.J_tensor.copy()
    bad[0, 1, 2] = np.inf
    assert _status(lambda: s.set_exchange_tensors(bad)) == "SLLG_E_ARG"
    sym = w.J_tensor.copy()
    sym[:] = 6e-21 * np.eye(3)               # symmetric tensors are their own transpose
    s.set_exchange_tensors(sym)
    s.set_exchange_tensors(None)
    s.set_materials([1.5 * 9.274e-24], [1e-23], [0, 0, 1.0], 0)
    assert _status(lambda: s.set_cubic_anisotropy([np.nan])) == "SLLG_E_ARG"
    s.set_cubic_anisotropy([2e-24])
    kc = np.linspace(-1e-24, 1e-24, w.n)
    s.set_cubic_anisotropy(kc)
    s.set_materials([1.5 * 9.274e-24], [1e-23], [0, 0, 1.0], 0)   # keeps the cubic constants
    s.set_cubic_anisotropy(None)
    # reverse links with a different type are accepted when their J agrees
    # (scalar exchange), and rejected when it does not
    J = np.array(w.J)
    J[1] *= 2
    assert _status(lambda: s.set_neighbours(lat.row_ptr, lat.col, lat.ntype, J)) == "SLLG_E_ARG"
    s.close()


def test_demag_and_relaxation_validation():
    w, s = _valid_system()
    lat = w.lattice
    pos = lat.pos * 0.3e-9
    assert _status(lambda: s.set_demag(pos, 0.6e-9, 2.7e-29, 10)) == "SLLG_E_STATE"   # no neighbours yet
    s.set_neighbours(lat.row_ptr, lat.col, lat.ntype, w.J)
    s.set_materials(w.mu_s[:1], w.k_u[:1], w.easy_axis[:1], 0)
    s.set_integrator(0.1, 1.76e11, 1e-16)
    s.set_conditions(0.0, (0.0, 0.0, 0.0))
    s.set_spins(w.S0)
    assert _status(lambda: s.demag_field()) == "SLLG_E_STATE"                        # not set
    assert _status(lambda: s.set_demag(pos, 0.0, 2.7e-29, 10)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_demag(pos, 0.6e-9, -1.0, 10)) == "SLLG_E_ARG"
    assert _status(lambda: s.set_demag(pos, 0.6e-9, 2.7e-29, 0)) == "SLLG_E_ARG"
    bad = pos.copy()
    bad[3, 1] = np.nan
    assert _status(lambda: s.set_demag(bad, 0.6e-9, 2.7e-29, 10)) == "SLLG_E_ARG"
    s.set_demag(pos, 0.6e-9, 2.7e-29, 10)
    assert _status(lambda: s.mc(5)) == "SLLG_E_STATE"          # Monte Carlo refuses the demagnetising field
    s.set_demag(None, 0, 0, 1)
    # relaxation arguments are checked before the device is touched
    assert _status(lambda: s.relax(-1.0, 10)) == "SLLG_E_ARG"
    assert _status(lambda: s.relax(1e-6, 10, check_every=0)) == "SLLG_E_ARG"
    s.set_conditions(300.0, (0.0, 0.0, 0.0))
    assert _status(lambda: s.relax(1e-6, 10)) == "SLLG_E_STATE"   # T > 0
    s.close()
