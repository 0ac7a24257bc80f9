"""GPU Monte Carlo (Hinzke-Nowak moves, colour-class sweeps) against the
oracle's Monte Carlo on the same inputs and the same counter-based draws.

In FP64 both sides take every acceptance decision in double precision from
the same random numbers, so the chains coincide (a decision could only
differ if a uniform fell within rounding of its acceptance probability):
spins, records and accepted counts are compared directly.  In FP32 the
decisions are the kernel's own, so the comparison is statistical.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import paper_1310_6143_amd as sl
from spin_systems import MU_B, bcc_block, fcc_nanoparticle, sc_reference
from spin_systems.lattice import Lattice
from spin_systems.workloads import GAMMA, Workload
from tests.gpu_util import angles, max_angle

pytestmark = pytest.mark.gpu
KB = 1.3807e-23


def _oracle_mc(w, n_steps):
    S = np.ascontiguousarray(w.S0.copy())
    m, E, acc = oracle.System(w).mc(S, 0, n_steps)
    return S, m, E, acc


@pytest.mark.parametrize("make", [lambda: sc_reference(L=12, temperature=300.0, seed=7),
                                  lambda: bcc_block(cells=10, temperature=900.0, seed=8),
                                  lambda: fcc_nanoparticle(radius_nm=1.6, temperature=300.0)])
def test_mc_fp64_chain_matches_oracle(make):
    w = make()
    S_ref, m_ref, E_ref, acc_ref = _oracle_mc(w, 25)
    with sl.from_workload(w, precision=sl.FP64, check_symmetry=False) as g:
        m, E, acc = g.mc(25)
        S = g.get_spins()
        assert g.step == 25
    assert np.array_equal(acc, acc_ref)
    assert max_angle(S, S_ref) <= 1e-12
    assert np.abs(m - m_ref).max() <= 1e-12
    assert np.abs(E - E_ref).max() <= 1e-12 * np.abs(E_ref).max()


def test_mc_chunked_equals_single_call_and_is_deterministic():
    w = sc_reference(L=10, temperature=500.0, seed=3)
    for prec in (sl.FP32, sl.FP64):
        with sl.from_workload(w, precision=prec) as a, sl.from_workload(w, precision=prec) as b:
            m1, E1, acc1 = a.mc(40)
            m2a, E2a, acc2a = b.mc(15)
            m2b, E2b, acc2b = b.mc(25)
            assert np.array_equal(a.get_spins(), b.get_spins())
            assert np.array_equal(m1, np.concatenate([m2a, m2b]))
            assert np.array_equal(acc1, np.concatenate([acc2a, acc2b]))


@pytest.mark.parametrize("T", [300.0, 400.0])
def test_mc_fp32_thermal_average_matches_oracle(T):
    w = sc_reference(L=12, temperature=T, seed=3)
    with sl.from_workload(w, precision=sl.FP32) as g:
        gpu = g.mc_average(1000, 3000, 10)
    ref, _ = oracle.mc_average(oracle.System(w), w.S0.copy(), 0, 1000, 3000, 10)
    # FP32 acceptance decisions differ from the oracle's where a uniform
    # falls within FP32 rounding of its probability, so the chains part and
    # agree in distribution: 3 combined blocked standard errors
    tol = 3 * np.hypot(gpu["m_abs_se"], ref["m_abs_se"])
    print(f"MC T={T}: gpu {gpu['m_abs']:.4f}+-{gpu['m_abs_se']:.4f} oracle {ref['m_abs']:.4f}+-{ref['m_abs_se']:.4f}")
    assert abs(gpu["m_abs"] - ref["m_abs"]) < tol, (gpu, ref)
    assert abs(gpu["acceptance"] - ref["acceptance"]) < 0.02


def test_mc_average_fp64_equals_oracle():
    """sllg_mc_average in FP64 runs the oracle's chain, so its averages are
    the oracle's up to the order of the FP64 sums; the accepted counts are
    the same integers."""
    w = sc_reference(L=8, temperature=500.0, seed=5)
    with sl.from_workload(w, precision=sl.FP64) as g:
        r = g.mc_average(200, 600, 6)
        assert g.step == 800
        # a second call continues the chain (step counter 800 onwards)
        r2 = g.mc_average(0, 300, 3)
    ref = oracle.System(w)
    S = w.S0.copy()
    o, step = oracle.mc_average(ref, S, 0, 200, 600, 6)
    o2, _ = oracle.mc_average(ref, S, step, 0, 300, 3)
    for a, b in ((r, o), (r2, o2)):
        assert abs(a["m_abs"] - b["m_abs"]) <= 1e-12
        assert abs(a["m_abs_se"] - b["m_abs_se"]) <= 1e-12
        assert np.abs(a["m"] - b["m"]).max() <= 1e-12
        assert abs(a["E"] - b["E"]) <= 1e-12 * abs(b["E"])
        assert abs(a["E_se"] - b["E_se"]) <= 1e-9 * abs(b["E"])
        assert a["acceptance"] == b["acceptance"]


def test_mc_average_rejects_bad_arguments():
    w = sc_reference(L=6, temperature=300.0, seed=5)
    with sl.from_workload(w, precision=sl.FP32) as g:
        for args in ((10, 0, 2), (-1, 10, 2), (10, 10, 1), (10, 10, 11)):
            with pytest.raises(sl.SllgError) as e:
                g.mc_average(*args)
            assert e.value.name == "SLLG_E_ARG"
        assert g.step == 0


@pytest.mark.parametrize("precision", [sl.FP32, sl.FP64])
def test_mc_boltzmann_ensemble_of_free_spins(precision):
    """4096 uncoupled anisotropic spins (k_u/kB T = 3): <cos^2 theta> over
    the ensemble and 400 steps against the Boltzmann integral."""
    n, ku, xi = 4096, 1e-23, 3.0
    lat = Lattice("free spins", np.zeros((n, 3)), np.zeros(n + 1, dtype=np.int64),
                  np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.uint8))
    w = Workload(name="free spins", lattice=lat, J=np.array([0.0]), mu_s=np.full(n, 1.5 * MU_B),
                 k_u=np.full(n, ku), easy_axis=np.tile([0.0, 0.0, 1.0], (n, 1)), alpha=0.1, gamma=GAMMA,
                 dt=1e-16, temperature=ku / (KB * xi), H=np.zeros(3), seed=17, n_steps=0,
                 S0=np.tile([0.0, 0.0, 1.0], (n, 1)))
    with sl.from_workload(w, precision=precision) as g:
        g.mc(200, record=False)
        samples = []
        for _ in range(40):
            g.mc(10, record=False)
            S = g.get_spins()
            samples.append((S[:, 2] ** 2).mean())
    samples = np.array(samples)
    num = integrate.quad(lambda t: np.cos(t) ** 2 * np.sin(t) * np.exp(xi * np.cos(t) ** 2), 0, np.pi)[0]
    den = integrate.quad(lambda t: np.sin(t) * np.exp(xi * np.cos(t) ** 2), 0, np.pi)[0]
    se = samples.std(ddof=1) / np.sqrt(samples.size)
    print(f"free spins: <cos^2> {samples.mean():.5f} +- {se:.5f}, Boltzmann {num / den:.5f}")
    assert abs(samples.mean() - num / den) < 3 * se, (samples.mean(), se, num / den)


def test_mc_chains_agree_bitwise_across_neighbour_forms():
    """Stencil and SELL rows list the same links in the same order (stencil
    padding adds J = 0 terms), and the Monte Carlo sum does not use the LDS
    window, so the chains agree bit for bit in every combination."""
    w = bcc_block(cells=12, temperature=700.0, seed=2)
    ref = None
    for stencil in (1, 0):
        for window in (1, 0):
            with sl.from_workload(w, precision=sl.FP32, stencil=stencil) as g:
                g.set_option("lds_window", window)
                m, E, acc = g.mc(30)
                S = g.get_spins()
            if ref is None:
                ref = (S, m, acc)
            else:
                assert np.array_equal(S, ref[0]) and np.array_equal(acc, ref[2]), (stencil, window)


def test_mc_longer_chain_in_two_calls_matches_oracle():
    """200 sweeps in two calls (136 + 64; the step counter continues) give
    the oracle's chain."""
    w = sc_reference(L=8, temperature=450.0, seed=12)
    S_ref, m_ref, E_ref, acc_ref = _oracle_mc(w, 200)
    with sl.from_workload(w, precision=sl.FP64) as g:
        m, E, acc = g.mc(136)
        m2, E2, acc2 = g.mc(64)
        S = g.get_spins()
        assert g.step == 200
    assert np.array_equal(np.concatenate([acc, acc2]), acc_ref)
    assert max_angle(S, S_ref) <= 1e-12
    assert np.abs(np.concatenate([m, m2]) - m_ref).max() <= 1e-12


def test_mc_full_block_in_the_bench_launch_shape():
    """The 8,192,000-spin bcc J1+J2 block as the benchmark runs it (default
    launch shape, 10 colour classes): FP64 chain identical to the oracle's
    over 2 steps at every site; FP32 after 1 step within 1e-4 rad of the
    oracle at all but a few sites (FP32 decisions can flip where the uniform
    falls within FP32 rounding of the acceptance probability, about one
    trial in 10^7, and a flipped site can tip a neighbour's later decision)."""
    w = bcc_block(cells=160)
    S_ref = np.ascontiguousarray(w.S0.copy())
    orc = oracle.System(w)
    m1, E1, acc1 = orc.mc(S_ref, 0, 1)
    S1 = S_ref.copy()
    m2, E2, acc2 = orc.mc(S_ref, 1, 1)
    m_ref, E_ref = np.concatenate([m1, m2]), np.concatenate([E1, E2])
    with sl.from_workload(w, precision=sl.FP64, check_symmetry=False) as g:
        assert g.get_option("fused_active") == 1   # records from the fused step's measuring walk
        m, E, acc = g.mc(2)
        S = g.get_spins()
    assert np.array_equal(acc, np.concatenate([acc1, acc2]))
    assert max_angle(S, S_ref) <= 1e-12
    # same spins; the records differ only by the order of their FP64 sums
    # over 8,192,000 sites, which the worst-case bound of a summation of N
    # terms, N 2^-53 = 9.1e-10 (relative), covers
    print(f"full block MC records: max |dm| {np.abs(m - m_ref).max():.2e}, "
          f"max |dE|/|E| {np.abs(E - E_ref).max() / np.abs(E_ref).max():.2e}")
    assert np.abs(m - m_ref).max() <= 1e-9
    assert np.abs(E - E_ref).max() <= 1e-9 * np.abs(E_ref).max()
    with sl.from_workload(w, precision=sl.FP32, check_symmetry=False) as g:
        m, E, acc = g.mc(1)
        S = g.get_spins()
    assert np.abs(m - m1).max() <= 1e-5
    assert np.abs(E - E1).max() <= 1e-5 * np.abs(E1).max()
    off = int((angles(S, S1) > 1e-4).sum())
    print(f"full block MC: FP64 accepted {acc1[0]} + {acc2[0]} as the oracle; FP32 step 1: "
          f"{off} of {w.n} sites off by more than 1e-4 rad, accepted {acc[0]} vs {acc1[0]}")
    assert off <= w.n // 10000
    assert abs(int(acc[0]) - int(acc1[0])) <= w.n // 10000


@pytest.mark.parametrize("stencil", [1, 0])
def test_mc_lattice_colouring_chain_matches_oracle(stencil):
    """Option "mc_colouring" = 1: the library colours the declared lattice in
    the visiting order grouped by basis site and cell parity, as the
    oracle's orc_lattice_visit does; the bcc J1+J2 block then has four
    colour classes (ten in ascending order) and the FP64 chain is the
    oracle's in that order, in both neighbour forms.  Back to 0, the chain
    is the ascending-order one again."""
    w = bcc_block(cells=10, temperature=900.0, seed=8)
    orc = oracle.System(w)
    S_ref = np.ascontiguousarray(w.S0.copy())
    m_ref, E_ref, acc_ref = orc.mc(S_ref, 0, 25, visit="lattice")
    S_asc = S_ref.copy()
    _, _, acc_asc = orc.mc(S_asc, 25, 10)
    with sl.from_workload(w, precision=sl.FP64, check_symmetry=False, stencil=stencil) as g:
        assert g.get_option("mc_colours") == int(orc.colours().max()) + 1
        g.set_option("mc_colouring", 1)
        assert g.get_option("mc_colouring") == 1
        assert g.get_option("mc_colours") == 4
        m, E, acc = g.mc(25)
        S = g.get_spins()
        g.set_option("mc_colouring", 0)
        _, _, acc2 = g.mc(10)
        S2 = g.get_spins()
    print(f"lattice-ordered colouring: 4 classes, accepted {acc.sum()} as the oracle")
    assert np.array_equal(acc, acc_ref)
    assert max_angle(S, S_ref) <= 1e-12
    assert np.abs(m - m_ref).max() <= 1e-12
    assert np.abs(E - E_ref).max() <= 1e-12 * np.abs(E_ref).max()
    assert np.array_equal(acc2, acc_asc)
    assert max_angle(S2, S_asc) <= 1e-12


def test_mc_lattice_colouring_without_a_lattice_is_ascending():
    """Without a lattice declaration the option leaves the ascending order."""
    w = bcc_block(cells=6, temperature=900.0, seed=9)
    S_ref = np.ascontiguousarray(w.S0.copy())
    _, _, acc_ref = oracle.System(w).mc(S_ref, 0, 10)
    with sl.from_workload(w, precision=sl.FP64, check_symmetry=False, lattice=False) as g:
        g.set_option("mc_colouring", 1)
        assert g.get_option("mc_colours") == int(oracle.System(w).colours().max()) + 1
        _, _, acc = g.mc(10)
        S = g.get_spins()
    assert np.array_equal(acc, acc_ref)
    assert max_angle(S, S_ref) <= 1e-12


def test_mc_full_block_lattice_colouring():
    """The 8,192,000-spin block with the four lattice-ordered classes, as the
    benchmark's Monte Carlo line runs it: one FP64 step identical to the
    oracle's at every site."""
    w = bcc_block(cells=160)
    S_ref = np.ascontiguousarray(w.S0.copy())
    m_ref, E_ref, acc_ref = oracle.System(w).mc(S_ref, 0, 1, visit="lattice")
    with sl.from_workload(w, precision=sl.FP64, check_symmetry=False) as g:
        g.set_option("mc_colouring", 1)
        assert g.get_option("mc_colours") == 4
        m, E, acc = g.mc(1)
        S = g.get_spins()
    print(f"full block, lattice-ordered classes: accepted {acc[0]} as the oracle; max |dm| "
          f"{np.abs(m - m_ref).max():.2e}, max |dE|/|E| {np.abs(E - E_ref).max() / np.abs(E_ref).max():.2e}")
    assert np.array_equal(acc, acc_ref)
    assert max_angle(S, S_ref) <= 1e-12
    # records: FP64 sums over 8,192,000 sites in another order (N 2^-53 = 9.1e-10)
    assert np.abs(m - m_ref).max() <= 1e-9
    assert np.abs(E - E_ref).max() <= 1e-9 * np.abs(E_ref).max()


def test_mc_colouring_option_is_validated():
    """"mc_colouring" takes 0 or 1 (anything else is SLLG_E_ARG and changes
    nothing); "mc_colours" reads the number of classes."""
    w = bcc_block(cells=4, temperature=300.0, seed=2)
    with sl.from_workload(w, precision=sl.FP32, check_symmetry=False) as g:
        before = g.get_option("mc_colours")
        with pytest.raises(sl.SllgError):
            g.set_option("mc_colouring", 2)
        assert g.get_option("mc_colouring") == 0
        assert g.get_option("mc_colours") == before
        g.set_option("mc_colouring", 1)
        assert g.get_option("mc_colours") == 4
