"""Pins for the oracle's tensorial exchange and cubic anisotropy (section on
the classical spin Hamiltonian: exchange as a 3x3 tensor whose off-diagonal
antisymmetric part is the Dzyaloshinskii-Moriya interaction; cubic
anisotropy (k_c/2)(Sx^4 + Sy^4 + Sz^4)), each against something other than
the oracle's own formulas:

- an isotropic tensor J * I reproduces the scalar-exchange trajectory bit
  for bit (the tensor form reduces to the scalar one);
- fields are the negative energy gradient, exactly: the energy is a
  polynomial of degree 4 in each spin's components, so the five-point
  derivative has no truncation error;
- a ring with exchange J and a Dzyaloshinskii-Moriya vector D along the
  ring relaxes at T = 0 to the flat spiral with turn angle
  theta = -atan(D/J) per bond and energy -n sqrt(J^2 + D^2) (closed form of
  the classical helix), with the handedness set by the sign of D; Monte
  Carlo at low temperature finds the same spiral energy;
- a single spin with cubic anisotropy relaxes to a <111> direction for
  k_c > 0 and to a <100> axis for k_c < 0 (the extrema of
  Sx^4 + Sy^4 + Sz^4 on the sphere), and samples the Boltzmann
  distribution exp(-(k_c/2)(Sx^4 + Sy^4 + Sz^4)/kB T), whose moments come
  from a two-dimensional quadrature over the sphere, under both Monte Carlo
  and the stochastic LLG integrator.
"""
import numpy as np
import pytest
from scipy import integrate

from spin_systems import MU_B, bcc, dmi_matrix, sc_reference, single_spin, with_tensor_exchange
from spin_systems.lattice import Lattice
from spin_systems.workloads import GAMMA, Workload

KB = 1.3807e-23


def _ring(n, J, D, temperature=0.0, alpha=1.0, dt=5e-16, seed=3, k_c=None):
    """n spins on a periodic chain along x; link i -> i+1 is type 0 with
    tensor J I - A(D x), the reverse link type 1 with the transpose."""
    i = np.arange(n)
    nxt, prv = (i + 1) % n, (i - 1) % n
    col = np.stack([prv, nxt], axis=1)
    typ = np.stack([np.ones(n), np.zeros(n)], axis=1)
    order = np.argsort(col, axis=1, kind="stable")
    col = np.take_along_axis(col, order, axis=1).astype(np.int32).ravel()
    typ = np.take_along_axis(typ, order, axis=1).astype(np.uint8).ravel()
    lat = Lattice(f"ring {n}", np.stack([i, 0 * i, 0 * i], 1).astype(float),
                  np.arange(0, 2 * n + 1, 2, dtype=np.int64), col, typ)
    fwd = J * np.eye(3) - dmi_matrix((D, 0.0, 0.0))
    w = Workload(name="dmi ring", lattice=lat, J=np.array([J, J]), mu_s=np.full(n, 1.5 * MU_B),
                 k_u=np.zeros(n), easy_axis=np.tile([0.0, 0.0, 1.0], (n, 1)), alpha=alpha, gamma=GAMMA,
                 dt=dt, temperature=temperature, H=np.zeros(3), seed=seed, n_steps=0,
                 S0=np.tile([0.0, 0.0, 1.0], (n, 1)), J_tensor=np.stack([fwd, fwd.T]))
    if k_c is not None:
        w.k_c = np.full(n, k_c)
    return w


def _spiral(n, theta, rng, noise):
    phi = theta * np.arange(n)
    S = np.stack([np.zeros(n), np.cos(phi), np.sin(phi)], 1) + noise * rng.standard_normal((n, 3))
    return np.ascontiguousarray(S / np.linalg.norm(S, axis=1, keepdims=True))


def _turn_angles(S):
    nxt = np.roll(S, -1, axis=0)
    return np.arctan2(np.cross(S, nxt)[:, 0], (S * nxt).sum(1))


def test_isotropic_tensor_equals_scalar_exchange(orc):
    w = sc_reference(L=6, temperature=300.0, seed=9)
    rng = np.random.default_rng(2)
    S0 = rng.standard_normal((w.n, 3))
    S0 /= np.linalg.norm(S0, axis=1, keepdims=True)
    a = S0.copy()
    m1, E1 = orc.System(w).integrate(a, 0, 200)
    w.J_tensor = np.array([6.0e-21 * np.eye(3)])
    b = S0.copy()
    m2, E2 = orc.System(w).integrate(b, 0, 200)
    assert np.array_equal(a, b) and np.array_equal(m1, m2) and np.array_equal(E1, E2)


def test_tensor_and_cubic_fields_are_negative_energy_gradient(orc):
    rng = np.random.default_rng(4)
    lat = bcc((3, 3, 3), (True, True, True), second_neighbours=True)
    n = lat.n
    base = Workload(name="random", lattice=lat, J=np.array([6e-21, 2.5e-21]),
                    mu_s=rng.uniform(1.0, 3.0, n) * MU_B, k_u=rng.uniform(0.0, 5e-23, n),
                    easy_axis=np.tile([0.0, 0.6, 0.8], (n, 1)), alpha=0.1, gamma=GAMMA, dt=1e-16,
                    temperature=0.0, H=np.array([0.3, -0.2, 0.7]), seed=5, n_steps=0,
                    S0=np.tile([0.0, 0.0, 1.0], (n, 1)))
    w = with_tensor_exchange(base, D=(1.5e-21, -0.7e-21), dmi="interfacial",
                             k_c=rng.uniform(-4e-22, 4e-22, n))
    # a general off-diagonal part as well: a symmetric traceless two-ion
    # term per shell (its own transpose, so the reverse link stays valid)
    B = np.array([[0.4, 0.3, -0.2], [0.3, -0.1, 0.5], [-0.2, 0.5, -0.3]])
    for t in range(w.J_tensor.shape[0]):
        w.J_tensor[t] += B * (1e-21 if w.J[t] == 6e-21 else -6e-22)
    s = orc.System(w)
    S = rng.standard_normal((n, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    H = s.fields(S)
    h = 1e-2
    for i in rng.choice(n, size=10, replace=False):
        for c in range(3):
            E = []
            for k in (-2, -1, 1, 2):
                Sk = S.copy()
                Sk[i, c] += k * h
                E.append(s.energy(Sk))
            grad = (E[0] - 8 * E[1] + 8 * E[2] - E[3]) / (12 * h)
            assert abs(-grad / w.mu_s[i] - H[i, c]) <= 1e-9 * np.abs(H[i]).max(), (i, c)


def test_reverse_links_carry_transposed_tensors():
    w = with_tensor_exchange(sc_reference(L=4), D=2e-21, dmi="bulk")
    lat = w.lattice
    rows = np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    for k in range(0, lat.nnz, 7):
        i, j, t = rows[k], lat.col[k], lat.ntype[k]
        q = lat.row_ptr[j] + np.nonzero(lat.col[lat.row_ptr[j]:lat.row_ptr[j + 1]] == i)[0][0]
        assert np.array_equal(w.J_tensor[lat.ntype[q]], w.J_tensor[t].T)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_dmi_ring_relaxes_to_the_helix(orc, sign):
    n, J = 16, 6.0e-21
    theta = -sign * 2 * np.pi / n                 # ground state: tan(theta) = -D/J
    D = -J * np.tan(theta)
    w = _ring(n, J, D)
    s = orc.System(w)
    S = _spiral(n, theta, np.random.default_rng(1), 0.15)
    assert s.relax(S, 1e-7, 2_000_000) >= 0
    ang = _turn_angles(S)
    assert np.abs(ang - theta).max() < 1e-7, (ang, theta)
    assert np.isclose(s.energy(S), -n * np.hypot(J, D), rtol=1e-12)
    # the uniform state carries no Dzyaloshinskii-Moriya energy
    up = np.tile([0.0, 0.0, 1.0], (n, 1))
    assert np.isclose(s.energy(up), -n * J, rtol=1e-14)


def test_mc_finds_the_helix_energy(orc):
    """At kB T << J the Monte Carlo energy is the helix ground state plus
    kB T per spin (two quadratic degrees of freedom each)."""
    n, J, T = 16, 6.0e-21, 2.0
    theta = -2 * np.pi / n
    D = -J * np.tan(theta)
    w = _ring(n, J, D, temperature=T)
    s = orc.System(w)
    S = _spiral(n, -theta, np.random.default_rng(5), 0.0)   # start from the wrong handedness
    s.mc(S, 0, 20000, record=False)
    _, E, _ = s.mc(S, 20000, 40000)
    mean, se = orc.block_stats(E, 20)
    expect = -n * np.hypot(J, D) + n * KB * T
    assert abs(mean - expect) < 4 * se + 0.05 * n * KB * T, (mean, expect, se)


@pytest.mark.parametrize("kc,target", [(1e-23, "111"), (-1e-23, "100")])
def test_cubic_ground_states(orc, kc, target):
    w = single_spin(k_u=0.0, alpha=1.0, dt=1e-14, S0=(0.9, 0.3, 0.5))
    w.k_c = np.array([kc])
    s = orc.System(w)
    S = w.S0.copy()
    assert s.relax(S, 1e-9, 5_000_000) >= 0
    a = np.sort(np.abs(S[0]))
    if target == "111":
        assert np.abs(a - 1 / np.sqrt(3)).max() < 1e-6, S
    else:
        assert abs(a[2] - 1.0) < 1e-9 and a[1] < 1e-4, S
    # energies at the extrema
    x = 0.5 * kc
    assert np.isclose(s.energy(np.array([[1.0, 0.0, 0.0]])), x, rtol=1e-14)
    assert np.isclose(s.energy(np.full((1, 3), 1 / np.sqrt(3))), x / 3, rtol=1e-14)


def _cubic_moment(xi):
    """<f> with f = Sx^4 + Sy^4 + Sz^4 under exp(-(xi/2) f) on the sphere."""
    def f(th, ph):
        st = np.sin(th)
        return (st * np.cos(ph)) ** 4 + (st * np.sin(ph)) ** 4 + np.cos(th) ** 4

    w = lambda th, ph: np.sin(th) * np.exp(-0.5 * xi * f(th, ph))
    num = integrate.dblquad(lambda th, ph: f(th, ph) * w(th, ph), 0, 2 * np.pi, 0, np.pi, epsabs=1e-12)[0]
    den = integrate.dblquad(w, 0, 2 * np.pi, 0, np.pi, epsabs=1e-12)[0]
    return num / den


@pytest.mark.parametrize("xi", [-6.0, 6.0])
def test_cubic_boltzmann_monte_carlo(orc, xi):
    kc, mu = 1e-23, 1.5 * MU_B
    T = abs(kc / (KB * xi))
    w = single_spin(mu_s=mu, k_u=0.0, temperature=T, S0=(0.6, 0.0, 0.8), seed=31)
    w.k_c = np.array([np.sign(xi) * kc])
    s = orc.System(w)
    S = w.S0.copy()
    s.mc(S, 0, 2000, record=False)
    m, _, _ = s.mc(S, 2000, 400_000)
    f = (m ** 4).sum(1)
    mean, se = orc.block_stats(f, 40)
    assert abs(mean - _cubic_moment(xi)) < 4 * se + 2e-3, (mean, se, _cubic_moment(xi))


def test_cubic_boltzmann_llg(orc):
    xi, kc, mu = 6.0, 1e-23, 1.5 * MU_B
    w = single_spin(mu_s=mu, k_u=0.0, alpha=1.0, dt=1e-14, temperature=kc / (KB * xi),
                    S0=(0.6, 0.0, 0.8), seed=32)
    w.k_c = np.array([kc])
    s = orc.System(w)
    S = w.S0.copy()
    s.integrate(S, 0, 20000, record=False)
    chunks, step = [], 20000
    for _ in range(3):
        m, _ = s.integrate(S, step, 1_000_000)
        step += 1_000_000
        chunks.append((m ** 4).sum(1))
    mean, se = orc.block_stats(np.concatenate(chunks), 40)
    assert abs(mean - _cubic_moment(xi)) < 4 * se + 2e-3, (mean, se, _cubic_moment(xi))
