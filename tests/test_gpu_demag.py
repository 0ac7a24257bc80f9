"""GPU macrocell demagnetising field against the oracle: the field itself
(cell moments, centres of mass, all-pairs dipole sum, self term) on shapes
with ragged surface cells, and integration with the update schedule across
chunk boundaries.
"""
import numpy as np
import pytest

import oracle
import paper_1310_6143_amd as sl
from spin_systems import (MU_B, GAMMA, Workload, fcc_ellipsoid, fcc_nanoparticle, simple_cubic,
                          with_demag)
from tests.gpu_util import max_angle

pytestmark = pytest.mark.gpu
MU0 = 4e-7 * np.pi


def _wl(lat, J=2.757e-21, mu=1.5 * MU_B, ku=0.0, T=0.0, alpha=0.1, dt=1e-16, seed=3, spread=0.4):
    n = lat.n
    rng = np.random.default_rng(seed)
    S0 = np.tile([0.0, 0.0, 1.0], (n, 1)) + spread * rng.standard_normal((n, 3))
    return Workload(name="demag", lattice=lat, J=np.array([J]), mu_s=np.full(n, mu), k_u=np.full(n, ku),
                    easy_axis=np.tile([0.0, 0.0, 1.0], (n, 1)), alpha=alpha, gamma=GAMMA, dt=dt, temperature=T,
                    H=np.array([0.0, 0.0, 0.2]), seed=seed, n_steps=0,
                    S0=S0 / np.linalg.norm(S0, axis=1, keepdims=True))


@pytest.mark.parametrize("shape", ["spheroid", "prism", "sphere_cells_2a"])
def test_demag_field_matches_oracle(shape):
    if shape == "spheroid":
        w = with_demag(_wl(fcc_ellipsoid(0.354, (2.5, 2.5, 5.0))), 0.354, 0.354, every=1)
    elif shape == "prism":
        w = with_demag(_wl(simple_cubic((31, 25, 7), (False, False, False))), 0.25, 0.75, every=1)
    else:   # partially filled surface cells, two unit cells per macrocell
        w = with_demag(_wl(fcc_nanoparticle(radius_nm=3.0).lattice), 0.3524, 0.7048, every=1)
    H_ref, n_cells = oracle.System(w).demag_field(w.S0)
    scale = np.abs(H_ref).max()
    for prec, tol in ((sl.FP64, 1e-12), (sl.FP32, 2e-5)):
        with sl.from_workload(w, precision=prec) as g:
            H = g.demag_field()
        err = np.abs(H - H_ref).max() / scale
        print(f"{shape} ({n_cells} cells) {'FP64' if prec == sl.FP64 else 'FP32'}: max rel error {err:.2e}")
        assert err <= tol


def test_integration_with_demag_matches_oracle():
    """Thermal dynamics of a ragged particle with the field updated every 7
    steps (updates fall inside and across the library's step chunks)."""
    base = fcc_nanoparticle(radius_nm=1.6, temperature=300.0)
    w = _wl(base.lattice, T=300.0)
    w.k_u, w.easy_axis = base.k_u, base.easy_axis
    w = with_demag(w, 0.3524, 0.3524, every=7)
    S_ref = np.ascontiguousarray(w.S0.copy())
    m_ref, E_ref = oracle.System(w).integrate(S_ref, 0, 500)
    with sl.from_workload(w, precision=sl.FP64) as g:
        m, E = g.integrate(500)
        S = g.get_spins()
    ang = max_angle(S, S_ref)
    print(f"integration with demag FP64: max angle {ang:.2e}")
    assert ang <= 1e-9
    assert np.abs(m - m_ref).max() <= 1e-10
    # chunked calls give the same result bit for bit (the schedule follows
    # the global step number)
    with sl.from_workload(w, precision=sl.FP64) as g:
        g.integrate(123, record=False)
        g.integrate(377, record=False)
        assert np.array_equal(g.get_spins(), S)
    with sl.from_workload(w, precision=sl.FP32) as g:
        g.integrate(500)
        assert max_angle(g.get_spins(), S_ref) <= 2e-3


def test_demag_field_at_benchmark_size_sampled():
    """The update the benchmark times: a simple-cubic slab of 128 x 128 x 32
    atoms (a = 0.25 nm) in macrocells of 2 atoms per edge (65,536 cells,
    8 source chunks of 8,192 cells), random spins; 512 sampled atoms against the oracle's
    per-cell evaluation.  FP32 bound: positions carry about 6e-8 of the
    32 nm slab (4e-6 of the nearest cell distance, tripled by 1/r^3) and each
    chunk sums 8,192 terms in FP32, about 2e-5 of the largest field in all;
    the bound is five times that."""
    lat = simple_cubic((128, 128, 32), (False, False, False))
    w = with_demag(_wl(lat, J=1e-21, spread=0.0), 0.25, 0.5, every=1)
    S = np.random.default_rng(1).standard_normal((w.n, 3))
    w.S0 = S / np.linalg.norm(S, axis=1, keepdims=True)
    sites = np.random.default_rng(2).choice(w.n, 512, replace=False)
    H_ref = oracle.System(w).demag_sample(w.S0, sites)
    scale = np.abs(H_ref).max()
    for prec, tol in ((sl.FP64, 1e-12), (sl.FP32, 1e-4)):
        with sl.from_workload(w, precision=prec) as g:
            H = g.demag_field()[sites]
        err = np.abs(H - H_ref).max() / scale
        print(f"65,536-cell slab {'FP64' if prec == sl.FP64 else 'FP32'}: max rel error {err:.2e} over 512 sites")
        assert err <= tol


def _demag_twin_case():
    base = fcc_nanoparticle(radius_nm=1.4, temperature=300.0)
    w = _wl(base.lattice, T=300.0)
    return with_demag(w, 0.3524, 0.3524, every=10)


@pytest.mark.parametrize("prec", [sl.FP64, sl.FP32])
def test_held_field_survives_autotune_checkpoint_and_reads(prec):
    """The field is updated every 10 steps and held in between.  At step 13
    (three steps into a hold) the autotuner, a checkpoint/restore into a
    fresh system and reading the field must each leave the spins bit for
    bit those of an untouched twin (the autotuner's tile size may move the
    m and E records at FP64 rounding)."""
    w = _demag_twin_case()
    with sl.from_workload(w, precision=prec) as twin, sl.from_workload(w, precision=prec) as a:
        twin.integrate(13, record=False)
        a.integrate(13, record=False)
        H_held = a.demag_field()
        assert np.array_equal(H_held, twin.demag_field())
        a.autotune(4)
        assert a.step == 13
        assert np.array_equal(a.demag_field(), H_held)
        blob = a.checkpoint()
        m_t, E_t = twin.integrate(24)
        S_t = twin.get_spins()
        m_a, E_a = a.integrate(24)
        assert np.array_equal(a.get_spins(), S_t)
        # the autotuner may pick another tile size: the records then move at FP64 rounding
        assert np.allclose(m_a, m_t, rtol=0, atol=1e-13) and np.allclose(E_a, E_t, rtol=1e-13, atol=0)
        with sl.from_workload(w, precision=prec) as b:
            b.restore(blob)
            assert b.step == 13
            assert np.array_equal(b.demag_field(), H_held)
            m_b, E_b = b.integrate(24)
            assert np.array_equal(b.get_spins(), S_t)
            assert np.array_equal(m_b, m_t) and np.array_equal(E_b, E_t)


def test_held_field_differs_from_field_of_current_spins():
    """Guards the test above: three steps into a hold the held field is not
    the field the current spins would give, so a recompute would be seen."""
    w = _demag_twin_case()
    with sl.from_workload(w, precision=sl.FP64) as a:
        a.integrate(13, record=False)
        H_held = a.demag_field()
        H_now, _ = oracle.System(w).demag_field(a.get_spins())
    assert np.abs(H_held - H_now).max() > 1e-9 * np.abs(H_now).max()
