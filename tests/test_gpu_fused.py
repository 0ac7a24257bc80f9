"""GPU parity of the fused plane-marching Heun step (one launch per step,
the predictor recomputed on a ring of cells around each workgroup's tile)
against the FP64 oracle, through the C ABI.

The fused step adds a site's exchange links in its own fixed order (links
into the plane below, its own plane, the plane above), so it agrees with
the oracle and with the two-launch step to rounding (FP32, or FP64 for the
simple-cubic and bcc kinds); the FP32 tolerances are about ten times the
differences measured on MI355X (printed on the lines starting "PARITY"),
the FP64 ones those of the two-launch FP64 step.  Spins do not depend on the tile
shape (each site's arithmetic is the same whichever workgroup computes it),
so different shapes must give bit-identical spins; the m and E records are
sums over items and may differ at FP64 rounding.
"""
import numpy as np
import pytest

import oracle
import paper_1310_6143_amd as sl
from spin_systems import bcc_block, bcc_film, sc_reference
from tests.gpu_util import max_angle, mean_angle, parity_report

pytestmark = pytest.mark.gpu


def _oracle_run(w, n_steps, step0=0):
    ref = oracle.System(w)
    S = np.ascontiguousarray(w.S0.copy())
    m, E = ref.integrate(S, step0, n_steps)
    return S, m, E


def _fused_system(w, shape=None, fused=2, precision=sl.FP32):
    g = sl.from_workload(w, precision=precision)
    g.set_option("fused", fused)
    if shape is not None:
        tx, ty, planes, threads = shape
        g.set_option("fused_tile_x", tx)
        g.set_option("fused_tile_y", ty)
        g.set_option("fused_planes", planes)
        g.set_option("fused_threads", threads)
    return g


def _run(w, n_steps, shape=None, fused=2, chunks=None, precision=sl.FP32):
    with _fused_system(w, shape, fused, precision) as g:
        assert g.get_option("fused_active") == (1 if fused else 0)
        if chunks is None:
            m, E = g.integrate(n_steps)
        else:
            parts = [g.integrate(c) for c in chunks]
            m = np.concatenate([p[0] for p in parts])
            E = np.concatenate([p[1] for p in parts])
        return g.get_spins(), m, E


def _sc_two_couplings(L=8):
    """sc L^3 whose z links have their own J: every site has the six
    simple-cubic links, but not one coupling per link slot, so the fused
    step reads the links from its generic pattern tables."""
    w = sc_reference(L=L)
    lat = w.lattice
    rows = np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    lat.ntype = (lat.pos[rows, 2] != lat.pos[lat.col, 2]).astype(np.uint8)
    w.J = np.array([6.0e-21, 3.0e-21])
    return w


def test_lattice_declared_for_crystals():
    """Crystals are declared cell by cell; below 2^20 spins the default runs
    the two-launch step, "fused" = 2 takes the fused step at any size (FP64:
    the compiled simple-cubic and bcc kinds only)."""
    for w in (sc_reference(L=8), bcc_block(cells=6, n_steps=10), bcc_film(nx=8, ny=8, nz=4)):
        for prec in (sl.FP32, sl.FP64):
            with sl.from_workload(w, precision=prec) as g:
                assert g.get_option("lattice") == 2
                assert g.get_option("fused_active") == 0
                g.set_option("fused", 2)
                assert g.get_option("fused_active") == 1
    w = _sc_two_couplings()
    with sl.from_workload(w, precision=sl.FP32) as g:
        g.set_option("fused", 2)
        assert g.get_option("fused_active") == 1
    with sl.from_workload(w, precision=sl.FP64) as g:
        g.set_option("fused", 2)
        assert g.get_option("fused_active") == 0
        with pytest.raises(sl.SllgError):
            g.set_option("fused_tile_x", 6)
            g.set_option("fused_tile_y", 6)
            g.set_option("fused_planes", 4)
            g.set_option("fused_threads", 256)


def test_generic_kind_fused_fp32_matches_oracle():
    w = _sc_two_couplings(L=12)
    w.temperature = 300.0
    S_ref, m_ref, E_ref = _oracle_run(w, 200)
    S, m, E = _run(w, 200)
    r = parity_report("fused sc 12^3 two couplings (generic kind) FP32 200 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 2e-5 and r["mean"] <= 5e-6
    assert r["dm"] <= 5e-7 and r["dE"] <= 1e-6


def test_sc4096_fused_fp32_matches_oracle():
    w = sc_reference(L=16, temperature=300.0, n_steps=1000, seed=42)
    S_ref, m_ref, E_ref = _oracle_run(w, 1000)
    S, m, E = _run(w, 1000)
    parity_report("fused sc 16^3 T=300 K FP32 1000 steps", S, S_ref, m, m_ref, E, E_ref)
    amax, amean = max_angle(S, S_ref), mean_angle(S, S_ref)
    dm = np.abs(m - m_ref).max()
    dE = (np.abs(E - E_ref) / np.abs(E_ref)).max()
    # measured 1.5e-6, 3.4e-7, 3.6e-8, 6.1e-8
    assert amax <= 2e-5 and amean <= 5e-6
    assert dm <= 5e-7 and dE <= 1e-6
    assert np.abs(np.linalg.norm(S, axis=1) - 1).max() <= 1e-6


def test_bcc_j1j2_fused_fp32_matches_oracle():
    w = bcc_block(cells=24, n_steps=300)
    w.H = np.array([0.3, -0.2, 0.5])
    S_ref, m_ref, E_ref = _oracle_run(w, 300)
    S, m, E = _run(w, 300)
    parity_report("fused bcc 24^3 J1+J2 FP32 300 steps", S, S_ref, m, m_ref, E, E_ref)
    amax, amean = max_angle(S, S_ref), mean_angle(S, S_ref)
    dm = np.abs(m - m_ref).max()
    dE = (np.abs(E - E_ref) / np.abs(E_ref)).max()
    # measured 7.8e-7, 1.7e-7, 3.4e-9, 1.7e-8
    assert amax <= 1e-5 and amean <= 2e-6
    assert dm <= 5e-8 and dE <= 2e-7


def test_film_open_z_fused_fp32_matches_oracle():
    # open z: the surface planes have their own link patterns
    w = bcc_film(nx=20, ny=12, nz=7, seed=5)
    w.temperature = 500.0
    w.H = np.array([0.0, 0.4, -0.3])
    S_ref, m_ref, E_ref = _oracle_run(w, 300)
    S, m, E = _run(w, 300)
    parity_report("fused film 20x12x7 open z FP32 300 steps", S, S_ref, m, m_ref, E, E_ref)
    amax, amean = max_angle(S, S_ref), mean_angle(S, S_ref)
    dm = np.abs(m - m_ref).max()
    # measured 1.1e-6, 1.7e-7, 2.9e-8
    assert amax <= 2e-5 and amean <= 2e-6
    assert dm <= 5e-7


def test_sc4096_fused_fp64_matches_oracle():
    w = sc_reference(L=16, temperature=300.0, n_steps=1000, seed=42)
    S_ref, m_ref, E_ref = _oracle_run(w, 1000)
    S, m, E = _run(w, 1000, precision=sl.FP64)
    r = parity_report("fused sc 16^3 T=300 K FP64 1000 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 1e-12 and r["mean"] <= 1e-13
    assert r["dm"] <= 1e-12 and r["dE"] <= 1e-12
    assert np.abs(np.linalg.norm(S, axis=1) - 1).max() <= 1e-15


def test_bcc_j1j2_fused_fp64_matches_oracle():
    w = bcc_block(cells=24, n_steps=300)
    w.H = np.array([0.3, -0.2, 0.5])
    S_ref, m_ref, E_ref = _oracle_run(w, 300)
    S, m, E = _run(w, 300, precision=sl.FP64)
    r = parity_report("fused bcc 24^3 J1+J2 FP64 300 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 1e-12 and r["mean"] <= 1e-13
    assert r["dm"] <= 1e-12 and r["dE"] <= 1e-12


def test_film_open_z_fused_fp64_matches_oracle():
    w = bcc_film(nx=20, ny=12, nz=7, seed=5)
    w.temperature = 500.0
    w.H = np.array([0.0, 0.4, -0.3])
    S_ref, m_ref, E_ref = _oracle_run(w, 300)
    S, m, E = _run(w, 300, precision=sl.FP64)
    r = parity_report("fused film 20x12x7 open z FP64 300 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 1e-12 and r["mean"] <= 1e-13
    assert r["dm"] <= 1e-12 and r["dE"] <= 1e-12


@pytest.mark.parametrize("make", [lambda: bcc_block(cells=20, n_steps=50),
                                  lambda: bcc_film(nx=26, ny=14, nz=9, seed=7),
                                  lambda: sc_reference(L=30, temperature=300.0, seed=9)])
def test_spins_independent_of_shape(make):
    """Tiles that divide the lattice or not, planes per item that divide
    the thickness or not, tiles wider than the lattice (the region wraps
    more than once), every block size: spins bit for bit the same."""
    w = make()
    w.temperature = 400.0
    shapes = [(6, 6, 4, 256), (14, 14, 10, 256), (30, 14, 7, 512), (20, 20, 16, 512), (62, 6, 5, 512),
              (40, 10, 64, 512), (30, 30, 9, 1024), (40, 22, 16, 1024)]
    ref = None
    for shp in shapes:
        S, m, E = _run(w, 20, shape=shp)
        if ref is None:
            ref = (S, m, E)
            continue
        assert np.array_equal(S, ref[0]), shp
        assert np.allclose(m, ref[1], rtol=0, atol=1e-12), shp
        assert np.allclose(E, ref[2], rtol=1e-12, atol=0), shp


@pytest.mark.parametrize("make", [lambda: bcc_block(cells=20, n_steps=50),
                                  lambda: bcc_film(nx=26, ny=14, nz=9, seed=7),
                                  lambda: sc_reference(L=30, temperature=300.0, seed=9)])
def test_spins_independent_of_shape_fp64(make):
    """FP64 shapes (rows of 16 sites for 256 threads, 32 for 512): spins bit
    for bit the same whatever the tile, planes per item and block size."""
    w = make()
    w.temperature = 400.0
    shapes = [(6, 6, 4, 256), (12, 16, 10, 256), (6, 20, 7, 256), (28, 14, 9, 512), (20, 17, 16, 512),
              (10, 17, 64, 512)]
    ref = None
    for shp in shapes:
        S, m, E = _run(w, 20, shape=shp, precision=sl.FP64)
        if ref is None:
            ref = (S, m, E)
            continue
        assert np.array_equal(S, ref[0]), shp
        assert np.allclose(m, ref[1], rtol=0, atol=1e-14), shp
        assert np.allclose(E, ref[2], rtol=1e-14, atol=0), shp


def test_fp64_shapes_out_of_range_rejected():
    """FP64: the region must fit a row of 16 (256 threads) or 32 (512)
    sites, and 1024 threads are not built."""
    w = bcc_block(cells=20, n_steps=10)
    for shp in ((14, 8, 4, 256), (30, 8, 4, 512), (20, 20, 4, 1024)):
        with _fused_system(w, precision=sl.FP64) as g:
            with pytest.raises(sl.SllgError):
                for key, v in zip(("fused_tile_x", "fused_tile_y", "fused_planes", "fused_threads"), shp):
                    g.set_option(key, v)


def test_chunked_equals_one_call_bitwise():
    w = bcc_block(cells=12, n_steps=50)
    S1, m1, E1 = _run(w, 37)
    S2, m2, E2 = _run(w, 37, chunks=[1, 2, 11, 23])
    assert np.array_equal(S1, S2)
    assert np.array_equal(m1, m2) and np.array_equal(E1, E2)


def test_fp64_chunked_equals_one_call_bitwise():
    w = bcc_block(cells=12, n_steps=50)
    S1, m1, E1 = _run(w, 37, precision=sl.FP64)
    S2, m2, E2 = _run(w, 37, chunks=[1, 2, 11, 23], precision=sl.FP64)
    assert np.array_equal(S1, S2)
    assert np.array_equal(m1, m2) and np.array_equal(E1, E2)


def test_fp64_fused_agrees_with_two_launch_step():
    w = bcc_block(cells=16, n_steps=30)
    Sf, mf, Ef = _run(w, 30, fused=2, precision=sl.FP64)
    St, mt, Et = _run(w, 30, fused=0, precision=sl.FP64)
    ang = max_angle(Sf, St)
    print(f"fused vs two-launch FP64, 30 steps: max angle {ang:.3e}")
    assert ang <= 1e-13
    assert np.abs(mf - mt).max() <= 1e-13
    assert (np.abs(Ef - Et) / np.abs(Et)).max() <= 1e-13


def test_fused_agrees_with_two_launch_step():
    w = bcc_block(cells=16, n_steps=30)
    Sf, mf, Ef = _run(w, 30, fused=2)
    St, mt, Et = _run(w, 30, fused=0)
    ang = max_angle(Sf, St)
    print(f"fused vs two-launch FP32, 30 steps: max angle {ang:.3e}")
    assert ang <= 1e-4
    assert np.abs(mf - mt).max() <= 1e-6
    assert (np.abs(Ef - Et) / np.abs(Et)).max() <= 1e-6


@pytest.mark.parametrize("lattice_cells", [16, 40])
def test_shape_change_between_calls(lattice_cells):
    """Changing the work-item shape between two calls (as the autotuner
    does) must re-list the items: the spins then follow the same trajectory
    as an untouched run, bit for bit."""
    w = bcc_block(cells=lattice_cells, n_steps=30)
    with _fused_system(w) as a, _fused_system(w) as b:
        a.integrate(10, record=False)
        for key, v in zip(("fused_tile_x", "fused_tile_y", "fused_planes", "fused_threads"), (14, 6, 5, 256)):
            a.set_option(key, v)
        assert a.get_option("fused_tile_x") == 14 and a.get_option("fused_threads") == 256
        a.integrate(10, record=False)
        # one field at a time, each intermediate shape valid
        for key, v in (("fused_threads", 1024), ("fused_planes", 9), ("fused_tile_y", 30), ("fused_tile_x", 30)):
            a.set_option(key, v)
        ma, Ea = a.integrate(10)
        b.integrate(20, record=False)
        mb, Eb = b.integrate(10)
        assert np.array_equal(a.get_spins(), b.get_spins())
        assert np.allclose(ma, mb, rtol=0, atol=1e-12) and np.allclose(Ea, Eb, rtol=1e-12, atol=0)


@pytest.mark.parametrize("precision", [sl.FP32, sl.FP64])
def test_records_do_not_change_the_spins(precision):
    """The step kernel built without the record code (launches where no
    replica records, and the first step of every call) computes the same
    spins bit for bit as the build with it: a run with records, one
    without, and one that switches between the two every call agree."""
    w = bcc_block(cells=12, n_steps=60)
    with _fused_system(w, precision=precision) as a, _fused_system(w, precision=precision) as b, \
            _fused_system(w, precision=precision) as c:
        assert a.get_option("fused_active") == 1
        a.integrate(30)
        b.integrate(30, record=False)
        for k in range(6):
            if k % 2:
                c.integrate(5)
            else:
                c.integrate(5, record=False)
        Sa, Sb, Sc = a.get_spins(), b.get_spins(), c.get_spins()
    assert np.array_equal(Sa, Sb)
    assert np.array_equal(Sa, Sc)
