"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs and the same Philox noise stream.

Tolerances (the per-spin angle is atan2(|a x b|, a.b)), about ten times
the differences measured on MI355X (each test prints its figures on a line
starting "PARITY"):
- FP64 GPU vs oracle: max angle <= 1e-12 rad after 1000 steps (measured
  up to 8e-15); the differences come only from FMA contraction and
  libm-vs-device transcendentals (~1 ulp).  Records: |dm| <= 1e-12 and
  |dE| <= 1e-13 |E| (measured 1e-13 and 2e-14; the sums over sites run in
  another order).
- FP32 GPU vs oracle, sc 16^3 over 1000 steps: max angle <= 2e-5 rad and
  mean angle <= 5e-6 rad (measured 1.5e-6 and 3.4e-7 at 300 K, 1.7e-6
  and 9.7e-7 at T = 0 in a field): FP32 rounding (~6e-8 per operation)
  accumulated over the steps.  Records: |dm| <= 1e-5, |dE| <= 5e-7 |E|.
"""
import numpy as np
import pytest

import oracle
import paper_1310_6143_amd as sl
from spin_systems import bcc_block, fcc_nanoparticle, sc_reference, bcc_film
from tests.gpu_util import max_angle, mean_angle, parity_report

pytestmark = pytest.mark.gpu


def _oracle_run(w, n_steps, step0=0):
    ref = oracle.System(w)
    S = np.ascontiguousarray(w.S0.copy())
    m, E = ref.integrate(S, step0, n_steps)
    return S, m, E


def _gpu_run(w, n_steps, precision, stencil=1, **opts):
    with sl.from_workload(w, precision=precision, stencil=stencil) as g:
        for k, v in opts.items():
            g.set_option(k, v)
        m, E = g.integrate(n_steps)
        return g.get_spins(), m, E


@pytest.mark.parametrize("step", [0, 7, (1 << 32) + 5])
def test_noise_stream_matches_oracle(step):
    n = 100_000
    ref = oracle.gaussians(42, step, np.arange(n))
    g64 = sl.thermal_normals(42, step, n, sl.FP64)
    assert np.abs(g64 - ref).max() < 1e-12
    g32 = sl.thermal_normals(42, step, n, sl.FP32)
    err = np.abs(g32 - ref)
    # hardware log2 / sin / cos in FP32: absolute error grows with |g|
    assert np.all(err <= 2e-5 * (1.0 + np.abs(ref))), err.max()


@pytest.mark.parametrize("stencil", [1, 0])
def test_sc4096_fp64_matches_oracle(stencil):
    w = sc_reference(L=16, temperature=300.0, n_steps=1000, seed=42)
    S_ref, m_ref, E_ref = _oracle_run(w, 1000)
    S, m, E = _gpu_run(w, 1000, sl.FP64, stencil=stencil)
    r = parity_report(f"sc 16^3 T=300 K FP64 stencil={stencil} 1000 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 1e-12 and r["mean"] <= 1e-13
    assert r["dm"] <= 1e-12 and r["dE"] <= 1e-13
    assert np.abs(np.linalg.norm(S, axis=1) - 1).max() <= 1e-15


def _tilted_in_field(L=16, seed=5):
    """sc L^3 at T = 0 from a tilted random state (spread 0.4 around
    (0.3, 0.1, 1)) in H = (0.4, -0.3, 1.2) T: every spin precesses and
    relaxes, and no noise enters, so the run checks the deterministic Heun
    step alone."""
    w = sc_reference(L=L, temperature=0.0, n_steps=1000, seed=42)
    rng = np.random.default_rng(seed)
    S0 = np.tile([0.3, 0.1, 1.0], (w.n, 1)) + 0.4 * rng.standard_normal((w.n, 3))
    w.S0 = S0 / np.linalg.norm(S0, axis=1, keepdims=True)
    w.H = np.array([0.4, -0.3, 1.2])
    return w


@pytest.mark.parametrize("precision", [sl.FP64, sl.FP32])
def test_sc4096_deterministic_tilted_in_field(precision):
    w = _tilted_in_field()
    S_ref, m_ref, E_ref = _oracle_run(w, 1000)
    assert max_angle(S_ref, w.S0) > 0.05           # the spins really moved
    S, m, E = _gpu_run(w, 1000, precision)
    name = "FP64" if precision == sl.FP64 else "FP32"
    r = parity_report(f"sc 16^3 T=0 tilted in field {name} 1000 steps", S, S_ref, m, m_ref, E, E_ref)
    if precision == sl.FP64:
        assert r["max"] <= 1e-12 and r["dm"] <= 1e-12 and r["dE"] <= 1e-13
    else:
        assert r["max"] <= 2e-5 and r["mean"] <= 1e-5
        assert r["dm"] <= 1e-5 and r["dE"] <= 5e-7


@pytest.mark.parametrize("fused", [2, 0])
def test_sc4096_fp32_within_stated_bound(fused):
    """The fused one-launch step and the two-launch step."""
    w = sc_reference(L=16, temperature=300.0, n_steps=1000, seed=42)
    S_ref, m_ref, E_ref = _oracle_run(w, 1000)
    S, m, E = _gpu_run(w, 1000, sl.FP32, fused=fused)
    r = parity_report(f"sc 16^3 T=300 K FP32 fused={fused} 1000 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 2e-5 and r["mean"] <= 5e-6
    assert r["dm"] <= 5e-7 and r["dE"] <= 5e-7
    assert np.abs(np.linalg.norm(S, axis=1) - 1).max() <= 1e-6


def test_ragged_sphere_per_site_axes_fp64():
    # a small fcc particle: ragged rows (3..12 neighbours), per-site materials
    # and random easy axes, spans several 512-site tiles and a partial one
    w = fcc_nanoparticle(radius_nm=1.6, temperature=300.0)
    w.H = np.array([0.2, -0.1, 0.5])
    assert w.n % 512 != 0 and w.n > 3 * 512
    S_ref, m_ref, E_ref = _oracle_run(w, 300)
    S, m, E = _gpu_run(w, 300, sl.FP64)
    r = parity_report(f"fcc sphere n={w.n} FP64 300 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 1e-12 and r["dm"] <= 1e-12 and r["dE"] <= 1e-13


def test_film_open_surfaces_fp64():
    w = bcc_film(nx=12, ny=10, nz=5)
    w.temperature = 500.0
    S_ref, m_ref, E_ref = _oracle_run(w, 300)
    S, m, E = _gpu_run(w, 300, sl.FP64)
    r = parity_report("bcc film 12x10x5 FP64 300 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 1e-12 and r["dm"] <= 1e-12 and r["dE"] <= 1e-13


def test_bcc_j1j2_32cubed_fp64():
    """The 32^3-cell periodic bcc J1+J2 system (65,536 spins) with the large
    block's parameters, 1000 steps against the oracle."""
    w = bcc_block(cells=32, n_steps=1000)
    S_ref, m_ref, E_ref = _oracle_run(w, 1000)
    S, m, E = _gpu_run(w, 1000, sl.FP64)
    r = parity_report("bcc 32^3 J1+J2 FP64 1000 steps", S, S_ref, m, m_ref, E, E_ref)
    # records: sums over 65,536 sites in another order
    assert r["max"] <= 1e-12 and r["dm"] <= 1e-11 and r["dE"] <= 5e-13


@pytest.mark.parametrize("make", [lambda: sc_reference(L=12, temperature=300.0, seed=2),
                                  lambda: bcc_film(nx=8, ny=6, nz=4, seed=3),
                                  lambda: bcc_block(cells=10, n_steps=100)])
def test_stencil_and_sell_layouts_agree_bitwise(make):
    """Both neighbour layouts list a row's near links (read from the LDS
    window) before its far ones, each part in CSR order, and add the two
    partial sums the same way, so trajectories are identical bit for bit."""
    w = make()
    w.temperature = 300.0
    for prec in (sl.FP32, sl.FP64):
        with sl.from_workload(w, precision=prec, stencil=1) as a, \
                sl.from_workload(w, precision=prec, stencil=0) as b:
            assert a.get_option("neighbour_format") == 1
            assert b.get_option("neighbour_format") == 0
            ma, Ea = a.integrate(150)
            mb, Eb = b.integrate(150)
            assert np.array_equal(a.get_spins(), b.get_spins())
            assert np.array_equal(ma, mb) and np.array_equal(Ea, Eb)


def test_chunked_equals_single_call_bitwise():
    w = sc_reference(L=12, temperature=300.0, seed=9)
    for prec in (sl.FP32, sl.FP64):
        with sl.from_workload(w, precision=prec) as a, sl.from_workload(w, precision=prec) as b:
            m1, E1 = a.integrate(1000)
            m2a, E2a = b.integrate(500)
            m2b, E2b = b.integrate(500)
            assert np.array_equal(a.get_spins(), b.get_spins())
            assert np.array_equal(m1, np.concatenate([m2a, m2b]))
            assert np.array_equal(E1, np.concatenate([E2a, E2b]))
            assert a.step == b.step == 1000


def test_graph_and_direct_launches_agree_bitwise():
    w = sc_reference(L=10, temperature=300.0, seed=3)
    out = []
    for gs in (0, 64, 16):
        with sl.from_workload(w, precision=sl.FP32) as g:
            g.set_option("graph_steps", gs)
            m, E = g.integrate(333)
            out.append((g.get_spins(), m, E))
    for S, m, E in out[1:]:
        assert np.array_equal(S, out[0][0])
        assert np.array_equal(m, out[0][1])
        assert np.array_equal(E, out[0][2])


def test_xcd_remap_does_not_change_results():
    w = sc_reference(L=20, temperature=300.0, seed=5)
    res = []
    for remap in (0, 1, 2):
        with sl.from_workload(w, precision=sl.FP32) as g:
            g.set_option("xcd_remap", remap)
            m, E = g.integrate(100)
            res.append((g.get_spins(), m, E))
    for other in res[1:]:
        assert np.array_equal(res[0][0], other[0])
        assert np.array_equal(res[0][1], other[1])
        assert np.array_equal(res[0][2], other[2])


def test_tile_order_does_not_change_results():
    """Plane-swept tile lists (any group width) only reorder the work: every
    tile's sums and the reduction tree are fixed by the tile index."""
    w = bcc_block(cells=32, n_steps=100)
    for prec in (sl.FP32, sl.FP64):
        res = []
        for order, group in ((0, 0), (1, 0), (1, 1), (1, 3)):
            with sl.from_workload(w, precision=prec, check_symmetry=False) as g:
                g.set_option("tile_order", order)
                g.set_option("tile_group", group)
                m, E = g.integrate(60)
                res.append((g.get_spins(), m, E))
        for other in res[1:]:
            assert np.array_equal(res[0][0], other[0])
            assert np.array_equal(res[0][1], other[1])
            assert np.array_equal(res[0][2], other[2])


@pytest.mark.parametrize("make", [lambda: bcc_block(cells=24, n_steps=100),
                                  lambda: fcc_nanoparticle(radius_nm=1.6, temperature=300.0)])
def test_lds_window_does_not_change_results(make):
    """Near neighbours through the LDS tile window or straight from global
    memory: the same terms in the same order, so the same bits."""
    w = make()
    for prec in (sl.FP32, sl.FP64):
        res = []
        for window in (1, 0):
            with sl.from_workload(w, precision=prec, check_symmetry=False) as g:
                g.set_option("lds_window", window)
                m, E = g.integrate(80)
                res.append((g.get_spins(), m, E))
        assert np.array_equal(res[0][0], res[1][0])
        assert np.array_equal(res[0][1], res[1][1]) and np.array_equal(res[0][2], res[1][2])


def test_tile_size_changes_only_record_rounding():
    """Spin updates never depend on the tiling; the m/E records differ only
    by the FP64 summation order of their first reduction level."""
    w = bcc_block(cells=24, n_steps=100)
    for prec, largest in ((sl.FP32, 2048), (sl.FP64, 1024)):
        res = []
        for tile in (0, 512, largest):
            with sl.from_workload(w, precision=prec, check_symmetry=False) as g:
                g.set_option("tile_sites", tile)
                assert g.get_option("tile_sites") == (tile or 512)
                m, E = g.integrate(80)
                res.append((g.get_spins(), m, E))
        for S, m, E in res[1:]:
            assert np.array_equal(S, res[0][0])
            assert np.allclose(m, res[0][1], rtol=0, atol=1e-13)
            assert np.allclose(E, res[0][2], rtol=1e-13, atol=0)


@pytest.mark.parametrize("L", [12, 64])
@pytest.mark.parametrize("lattice", [False, True])
def test_autotune_leaves_trajectory_unchanged(L, lattice):
    """Two-launch step (no lattice declaration) and fused step (lattice
    declared): spins bit for bit; the records are FP64 sums of per-tile or
    per-workgroup partial sums, so a different tile size or shape may move
    them at FP64 rounding."""
    w = sc_reference(L=L, temperature=300.0, seed=13)
    with sl.from_workload(w, precision=sl.FP32, lattice=lattice) as a, \
            sl.from_workload(w, precision=sl.FP32, lattice=lattice) as b:
        if lattice:   # the fused step at these sizes
            a.set_option("fused", 2)
            b.set_option("fused", 2)
        a.integrate(7, record=False)
        b.integrate(7, record=False)
        us, choice = a.autotune(8)
        assert us > 0
        if lattice:
            assert a.get_option("fused_active") == 1
            assert choice["fused_tile_x"] > 0 and choice["fused_threads"] in (256, 512, 1024)
        else:
            assert choice["grid_scale_pct"] in (50, 100, 200) and choice["tile_sites"] in (512, 1024, 2048)
        assert a.step == b.step == 7
        ma, Ea = a.integrate(100)
        mb, Eb = b.integrate(100)
        assert np.array_equal(a.get_spins(), b.get_spins())
        assert np.allclose(ma, mb, rtol=0, atol=1e-13) and np.allclose(Ea, Eb, rtol=1e-13, atol=0)


def test_run_to_run_determinism():
    w = sc_reference(L=16, temperature=300.0, seed=42)
    a = _gpu_run(w, 200, sl.FP32)
    b = _gpu_run(w, 200, sl.FP32)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_checkpoint_resume_is_exact():
    w = sc_reference(L=8, temperature=300.0, seed=11)
    with sl.from_workload(w, precision=sl.FP64) as a:
        a.integrate(500, record=False)
        blob = a.checkpoint()
        m_cont, E_cont = a.integrate(500)
        S_cont = a.get_spins()
    with sl.from_workload(w, precision=sl.FP64) as b:
        b.restore(blob)
        assert b.step == 500
        m_res, E_res = b.integrate(500)
        assert np.array_equal(b.get_spins(), S_cont)
        assert np.array_equal(m_res, m_cont) and np.array_equal(E_res, E_cont)


def test_measure_initial_state_closed_form():
    w = sc_reference(L=8)
    w.H = np.array([0.0, 0.0, 0.3])
    with sl.from_workload(w, precision=sl.FP64) as g:
        m, E = g.measure()
    links = w.lattice.nnz // 2
    expect = -links * 6e-21 - w.n * 1e-23 - w.n * w.mu_s[0] * 0.3
    assert np.allclose(m, [0, 0, 1], atol=1e-15)
    assert np.isclose(E, expect, rtol=1e-13)


def test_average_matches_oracle():
    w = sc_reference(L=8, temperature=400.0, seed=21)
    with sl.from_workload(w, precision=sl.FP64) as g:
        r = g.average(300, 1000, 10)
    ref = oracle.System(w)
    S = w.S0.copy()
    o, _ = oracle.average(ref, S, 0, 300, 1000, 10)
    assert abs(r["m_abs"] - o["m_abs"]) < 1e-8
    assert abs(r["m_abs_se"] - o["m_abs_se"]) < 1e-8
    assert np.allclose(r["m"], o["m"], atol=1e-8)
    assert abs(r["E"] - o["E"]) < 1e-8 * abs(o["E"])


def test_temperature_sweep_continuation_matches_oracle():
    w = sc_reference(L=6, seed=8)
    temps = [0.0, 200.0, 600.0]
    with sl.from_workload(w, precision=sl.FP64) as g:
        rows = g.sweep_temperature(temps, 100, 200, 4)
        step = g.step
    ref = oracle.System(w)
    S = w.S0.copy()
    orows, ostep = oracle.sweep_temperature(ref, S, temps, 100, 200, 0, 4)
    assert step == ostep
    for a, b in zip(rows, orows):
        assert abs(a["m_abs"] - b["m_abs"]) < 1e-8
        assert abs(a["E"] - b["E"]) < 1e-8 * abs(b["E"])


def test_field_sweep_matches_oracle():
    w = sc_reference(L=6, seed=8, temperature=50.0)
    fields = [[0, 0, -2.0], [0, 0, 0.0], [0, 0, 2.0]]
    with sl.from_workload(w, precision=sl.FP64) as g:
        rows = g.sweep_field(fields, 100, 200, 4)
    ref = oracle.System(w)
    S = w.S0.copy()
    orows, _ = oracle.sweep_field(ref, S, fields, 100, 200, 0, 4)
    for a, b in zip(rows, orows):
        assert np.allclose(a["m"], b["m"], atol=1e-8)
