"""GPU parity at the edges: degenerate systems (one spin, two spins),
ragged sizes that end mid-wavefront and mid-tile, the full 8,192,000-spin
bcc block in the launch configuration bench.py times, and the largest system
the library accepts (2^28 - 1 spins).  Everything is checked
against the FP64 oracle on the same inputs and noise stream.
"""
import numpy as np
import pytest

import oracle
import paper_1310_6143_amd as sl
from spin_systems import bcc_block, sc_reference, single_spin
from spin_systems.lattice import Lattice
from spin_systems.workloads import GAMMA, MU_B, Workload
from tests.gpu_util import max_angle, parity_report

pytestmark = pytest.mark.gpu


def _oracle(w, n_steps):
    S = np.ascontiguousarray(w.S0.copy())
    m, E = oracle.System(w).integrate(S, 0, n_steps)
    return S, m, E


def _gpu(w, n_steps, precision, **opts):
    with sl.from_workload(w, precision=precision) as g:
        for k, v in opts.items():
            g.set_option(k, v)
        m, E = g.integrate(n_steps)
        return g.get_spins(), m, E


def _ring(n, temperature=300.0, seed=5, J=6.0e-21):
    """A periodic chain of n spins (two neighbours each), tilted start."""
    i = np.arange(n)
    col = np.stack([(i - 1) % n, (i + 1) % n], axis=1).astype(np.int32).ravel()
    row_ptr = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    lat = Lattice(f"ring {n}", np.stack([i, 0 * i, 0 * i], axis=1).astype(float), row_ptr, col,
                  np.zeros(2 * n, dtype=np.uint8))
    rng = np.random.default_rng(n)
    S0 = np.tile([0.0, 0.0, 1.0], (n, 1)) + 0.3 * rng.standard_normal((n, 3))
    S0 /= np.linalg.norm(S0, axis=1, keepdims=True)
    return Workload(name=f"ring {n}", lattice=lat, J=np.array([J]), mu_s=np.full(n, 1.5 * MU_B),
                    k_u=np.full(n, 1e-23), easy_axis=np.tile([0.0, 0.0, 1.0], (n, 1)), alpha=0.1,
                    gamma=GAMMA, dt=1e-16, temperature=temperature, H=np.array([0.0, 0.2, -0.5]),
                    seed=seed, n_steps=200, S0=S0)


@pytest.mark.parametrize("temperature", [0.0, 300.0])
def test_single_spin(temperature):
    """One spin, no neighbours: anisotropy, field and noise only."""
    w = single_spin(k_u=1e-23, H=(0.5, 0.0, 2.0), temperature=temperature, S0=(1.0, 0.2, 0.1),
                    seed=9, dt=1e-16, n_steps=2000)
    S_ref, m_ref, E_ref = _oracle(w, 2000)
    S, m, E = _gpu(w, 2000, sl.FP64)
    r = parity_report(f"single spin T={temperature} FP64 2000 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 1e-13 and r["dm"] <= 1e-13 and r["dE"] <= 1e-13   # measured <= 1e-14
    S32, m32, E32 = _gpu(w, 2000, sl.FP32)
    r = parity_report(f"single spin T={temperature} FP32 2000 steps", S32, S_ref, m32, m_ref, E32, E_ref)
    assert r["max"] <= 2e-5 and r["dm"] <= 2e-5 and r["dE"] <= 1e-5     # measured <= 2.3e-6


@pytest.mark.parametrize("n", [3, 63, 65, 511, 513, 2047, 2049, 4097])
def test_ragged_ring_sizes(n):
    """Systems ending mid-wavefront and mid-tile (tiles of 512 sites here)."""
    w = _ring(n)
    S_ref, m_ref, E_ref = _oracle(w, 200)
    S, m, E = _gpu(w, 200, sl.FP64)
    r = parity_report(f"ring {n} FP64 200 steps", S, S_ref, m, m_ref, E, E_ref)
    assert r["max"] <= 1e-13 and r["dm"] <= 1e-12 and r["dE"] <= 1e-13   # measured <= 3.5e-15, 1e-13, 6e-15
    S32, m32, E32 = _gpu(w, 200, sl.FP32)
    r = parity_report(f"ring {n} FP32 200 steps", S32, S_ref, m32, m_ref, E32, E_ref)
    assert r["max"] <= 2e-5 and r["mean"] <= 5e-6                        # measured <= 1.5e-6, 3.3e-7
    assert r["dm"] <= 5e-6 and r["dE"] <= 5e-6                           # measured <= 2.4e-7, 4.7e-7


def test_full_size_block_matches_oracle():
    """The 8,192,000-spin bcc J1+J2 block at its real size and in the launch
    configurations the benchmark runs: 3 steps against the oracle (every
    site)."""
    w = bcc_block(cells=160, n_steps=3)
    rng = np.random.default_rng(11)
    S0 = np.tile([0.0, 0.0, 1.0], (w.n, 1)) + 0.1 * rng.standard_normal((w.n, 3))
    w.S0 = S0 / np.linalg.norm(S0, axis=1, keepdims=True)
    S_ref, m_ref, E_ref = _oracle(w, 3)
    # m and E are sums over 8.2M sites: the oracle adds them one by one, the
    # GPU as a tree, so FP64 records agree to about N * eps = 2e-9 at worst
    # The fused step in the library's default shape and in the shape the
    # autotuner picks on the benchmark box, and the two-launch step, in both
    # precisions (measured: FP64 3.4e-16 rad, |dm| 1.2e-11; FP32 4.5e-6 rad
    # at one site, mean 1.2e-8, |dm| and |dE|/|E| 3.7e-9)
    runs = ((sl.FP64, 1, None, 1e-13, 1e-10, 1e-12), (sl.FP64, 1, (27, 15, 23, 512), 1e-13, 1e-10, 1e-12),
            (sl.FP64, 0, None, 1e-13, 1e-10, 1e-12), (sl.FP32, 1, None, 1e-5, 5e-8, 5e-8),
            (sl.FP32, 1, (40, 10, 20, 512), 1e-5, 5e-8, 5e-8), (sl.FP32, 0, None, 1e-5, 5e-8, 5e-8))
    fused_spins = {}
    for prec, fused, shape, ang_tol, m_tol, e_tol in runs:
        with sl.from_workload(w, precision=prec, check_symmetry=False) as g:
            g.set_option("fused", fused)
            if shape:
                for key, v in zip(("fused_tile_x", "fused_tile_y", "fused_planes", "fused_threads"), shape):
                    g.set_option(key, v)
            assert g.get_option("fused_active") == fused
            if not fused:
                assert g.get_option("tile_sites") == (2048 if prec == sl.FP32 else 1024)
            m, E = g.integrate(3)
            S = g.get_spins()
        label = f"full bcc block {'FP32' if prec == sl.FP32 else 'FP64'} fused={fused} shape={shape} 3 steps"
        ang = parity_report(label, S, S_ref, m, m_ref, E, E_ref)["max"]
        if fused:
            if prec not in fused_spins:
                fused_spins[prec] = S
            else:
                assert np.array_equal(S, fused_spins[prec])     # spins do not depend on the fused shape
        assert ang <= ang_tol
        assert np.abs(m - m_ref).max() <= m_tol
        assert np.abs(E - E_ref).max() <= e_tol * np.abs(E_ref).max()


# measured: FP32 1.0e-7 rad, FP64 2.1e-16 rad
@pytest.mark.parametrize("precision,tol", [(sl.FP32, 1e-6), (sl.FP64, 1e-14)])
def test_maximum_size_ring(precision, tol):
    """The largest system the C ABI accepts, 2^28 - 1 spins, as a ring: spin
    byte offsets pass 2^31 (so the rows take the SELL form), and the last
    tile is ragged.  One step at T = 0 from a twisted state; 1024
    sampled sites (both ends and the middle among them) against the oracle
    on the 5-site open chain around each: a site's Heun step reads its own
    and its neighbours' predictors, which read one site further, so the
    chain's middle site is exact.  The step's m record against the mean of
    the returned spins."""
    n = (1 << 28) - 1
    J, mu, ku, H = 6.0e-21, 1.5 * MU_B, 1e-23, np.array([0.3, -0.2, 0.5])
    axis = np.array([0.0, 0.6, 0.8])

    def state(i):
        i = np.asarray(i, dtype=np.float64)
        th = 0.6 + 0.4 * np.sin(0.013 * i)
        ph = 0.37 * i
        return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=-1)

    g = sl.SpinSystem(n, precision)
    try:
        g.set_option("check_symmetry", 0)
        i = np.arange(n, dtype=np.int64)
        col = np.empty(2 * n, dtype=np.int32)
        col[0::2] = (i - 1) % n
        col[1::2] = (i + 1) % n
        del i
        g.set_neighbours(np.arange(0, 2 * n + 1, 2, dtype=np.int64), col, None, [J])
        del col
        assert g.get_option("neighbour_format") == 0          # SELL: the stencil needs offsets below 2^31 bytes
        g.set_materials([mu], [ku], axis, per_site=0)
        g.set_integrator(0.1, GAMMA, 1e-16)
        g.set_conditions(0.0, H)
        g.set_rng(1, 0)
        g.set_spins(state(np.arange(n)))
        m, _ = g.integrate(1)
        S = g.get_spins()
    finally:
        g.close()
    rng = np.random.default_rng(11)
    sites = np.concatenate([[0, 1, 2, n // 2, (1 << 27) + 5, n - 3, n - 2, n - 1],
                            rng.integers(0, n, 1016)])
    k = sites.size
    # k disjoint open chains of 5 sites, centre at local index 2
    loc = np.arange(5 * k).reshape(k, 5)
    rows = [[] for _ in range(5 * k)]
    for a, b in zip(loc[:, :-1].ravel(), loc[:, 1:].ravel()):
        rows[a].append(b)
        rows[b].append(a)
    row_ptr = np.zeros(5 * k + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    ccol = np.array([c for r in rows for c in sorted(r)], dtype=np.int32)
    lat = Lattice("chains", np.zeros((5 * k, 3)), row_ptr, ccol, np.zeros(ccol.size, dtype=np.uint8))
    S0 = state((sites[:, None] + np.arange(-2, 3)[None, :]) % n).reshape(-1, 3)
    S0 /= np.linalg.norm(S0, axis=1, keepdims=True)
    w = Workload(name="chains", lattice=lat, J=np.array([J]), mu_s=np.full(5 * k, mu), k_u=np.full(5 * k, ku),
                 easy_axis=np.tile(axis, (5 * k, 1)), alpha=0.1, gamma=GAMMA, dt=1e-16, temperature=0.0, H=H,
                 seed=1, n_steps=1, S0=S0)
    S_ref = np.ascontiguousarray(S0.copy())
    oracle.System(w).integrate(S_ref, 0, 1, record=False)
    ang = max_angle(S[sites], S_ref[loc[:, 2]])
    dm = np.abs(m[0] - S.mean(axis=0)).max()
    name = "FP32" if precision == sl.FP32 else "FP64"
    print(f"ring of {n} spins {name}: max angle {ang:.2e} over {k} sampled sites; |m - mean S| {dm:.1e}")
    assert ang <= tol
    assert dm <= 1e-9


def test_undamped_dynamics_and_zero_steps():
    """lambda = 0, the method's degenerate damping: the thermal width
    vanishes with lambda, so the run is noise-free even at 300 K.  FP64 vs
    the oracle over 1000 steps from a tilted random state with anisotropy and
    a field along z: spins, m and E (whose drift is then the Heun scheme's
    alone, the same on both sides).  integrate(0) changes nothing."""
    w = sc_reference(L=8, temperature=300.0, alpha=0.0, dt=1e-16)
    rng = np.random.default_rng(21)
    S0 = np.tile([0.0, 0.0, 1.0], (w.n, 1)) + 0.5 * rng.standard_normal((w.n, 3))
    w.S0 = S0 / np.linalg.norm(S0, axis=1, keepdims=True)
    w.H = np.array([0.0, 0.0, 0.4])
    S_ref, m_ref, E_ref = _oracle(w, 1000)
    with sl.from_workload(w, precision=sl.FP64) as g:
        m0, E0 = g.integrate(0)
        assert m0.shape == (0, 3) and E0.shape == (0,) and g.step == 0
        assert np.abs(g.get_spins() - w.S0).max() <= 1e-15
        m, E = g.integrate(1000)
        S = g.get_spins()
    r = parity_report("lambda = 0 FP64 1000 steps", S, S_ref, m, m_ref, E, E_ref)
    print(f"lambda = 0 FP64: E drift {E[-1] - E[0]:.3e} J (oracle {E_ref[-1] - E_ref[0]:.3e})")
    assert r["max"] <= 5e-13 and r["dm"] <= 1e-13 and r["dE"] <= 1e-13   # measured 2.3e-14, 2.8e-15, 2.2e-15


def test_large_steps_keep_parity():
    """Steps that turn a spin by a large angle (fields of 1000 T and more
    with the exchange, dt = 2 fs: gamma |H| dt of 0.35 to 1.3 rad): the
    corrector rebuilds S + dS dt/2 from S and the normalised predictor
    through S.S' = 1/|S + dS dt|, which is then far from 1.  FP64 and FP32
    against the oracle's direct form over 100 steps at 300 K."""
    w = sc_reference(L=8, temperature=300.0, alpha=0.1, dt=2e-15)
    rng = np.random.default_rng(31)
    S0 = np.tile([0.0, 0.0, 1.0], (w.n, 1)) + 0.7 * rng.standard_normal((w.n, 3))
    w.S0 = S0 / np.linalg.norm(S0, axis=1, keepdims=True)
    w.H = np.array([300.0, 0.0, 950.0])
    S_ref, m_ref, E_ref = _oracle(w, 100)
    # measured: FP64 1.5e-14 rad, FP32 8.1e-6 rad (|dm| 2.3e-15, 6.1e-8)
    for prec, tol in ((sl.FP64, 2e-13), (sl.FP32, 1e-4)):
        S, m, E = _gpu(w, 100, prec)
        r = parity_report(f"large steps {'FP64' if prec == sl.FP64 else 'FP32'} 100 steps", S, S_ref, m, m_ref,
                          E, E_ref)
        assert r["max"] <= tol
        assert r["dm"] <= (1e-13 if prec == sl.FP64 else 1e-6)


def test_non_finite_spins_are_reported():
    """A field too large for the arithmetic (finite, 1e300 T) drives the
    spins to NaN: every new spin is checked by the kernel that writes it, so
    the asynchronous device-record path reports it too (at the next call,
    once the earlier work is done), sllg_integrate at its end; new spins
    clear the flag."""
    for prec in (sl.FP32, sl.FP64):
        w = sc_reference(L=8, temperature=0.0, n_steps=5)
        w.H = np.array([1e300, 0.0, 0.0])
        with sl.from_workload(w, precision=prec) as g:
            assert g.get_option("numeric_fault") == 0
            g.integrate_dev(3)
            assert g.get_option("numeric_fault") == 1      # waits for the queued steps
            with pytest.raises(sl.SllgError) as e:
                g.integrate_dev(1)
            assert e.value.name == "SLLG_E_NUMERIC"
            g.set_spins(w.S0)
            assert g.get_option("numeric_fault") == 0
            with pytest.raises(sl.SllgError) as e:
                g.integrate(2, record=False)
            assert e.value.name == "SLLG_E_NUMERIC"
            g.set_spins(w.S0)
            g.set_conditions(0.0, (0.0, 0.0, 1.0))
            g.integrate_dev(3)
            g.integrate_dev(3)                             # no fault: the call goes through
            assert g.get_option("numeric_fault") == 0
