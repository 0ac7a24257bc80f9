"""Pins for the oracle's Monte Carlo ("Monte Carlo Methods": Metropolis
acceptance, Hinzke-Nowak flip / Gaussian / random trial moves), each against
something other than the oracle's own formulas:

- the colouring is proper (no link inside a colour class) and greedy, by
  brute force over every link;
- the move choice and the acceptance uniform have the distributions the
  counter layout promises;
- a single spin samples the Boltzmann distribution: with uniaxial
  anisotropy the <cos^2 theta> integral ("Boltzmann distribution for a
  single spin"), in an applied field the Langevin function coth x - 1/x;
- at T = 0 no accepted trial raises the energy;
- the paper's simple-cubic M(T) fit (Tc = 631.82 K, beta = 0.334297 for
  J = 6.0e-21 J/link) and agreement with the stochastic LLG oracle at the
  same temperature (the paper's Monte Carlo vs LLG comparison);
- the colour-class sweep order (the one the GPU kernel takes) samples the
  same equilibrium as the paper's order (N trials on random sites), below,
  near and above Tc;
- the lattice visiting order of the colouring (basis site, cell parity)
  groups the sites as the builder placed them, gives the bcc J1+J2 lattice
  four equal proper classes, and its chain samples the same equilibrium as
  the random-site chain.
"""
import os
from multiprocessing import get_context

import numpy as np
import pytest
from scipy import integrate, stats

from spin_systems import MU_B, bcc, bcc_block, bcc_film, fcc_nanoparticle, sc_reference, simple_cubic, single_spin

KB = 1.3807e-23


def _check_colouring(orc, row_ptr, col):
    colour, k = orc.greedy_colours(row_ptr, col)
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    assert np.all(colour[rows] != colour[col]), "a link joins two sites of one colour"
    assert colour.min() >= 0 and colour.max() == k - 1
    # greedy: every smaller colour is taken by an earlier neighbour
    for i in range(min(n, 3000)):
        nb = col[row_ptr[i]:row_ptr[i + 1]]
        taken = set(colour[nb[nb < i]].tolist())
        assert all(c in taken for c in range(colour[i]))
    return k


def test_colouring_is_proper_and_greedy(orc):
    sc = simple_cubic((6, 6, 6), (True, True, True))
    assert _check_colouring(orc, sc.row_ptr, sc.col) == 2    # even periodic sc: a checkerboard
    b = bcc((4, 4, 4), (True, True, True), second_neighbours=True)
    k = _check_colouring(orc, b.row_ptr, b.col)
    assert k <= 15
    f = bcc_film(nx=6, ny=6, nz=4).lattice
    _check_colouring(orc, f.row_ptr, f.col)
    s = fcc_nanoparticle(radius_nm=1.2).lattice
    _check_colouring(orc, s.row_ptr, s.col)


def test_move_choice_and_acceptance_uniform(orc):
    draws = [orc.mc_choice(7, 123, i) for i in range(60000)]
    moves = np.array([d[0] for d in draws])
    u = np.array([d[1] for d in draws])
    counts = np.bincount(moves, minlength=3)
    assert counts.size == 3
    assert stats.chisquare(counts).pvalue > 1e-4
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    assert u.min() >= 0.0 and u.max() < 1.0
    # the move choice and the uniform are independent
    assert abs(np.corrcoef(moves, u)[0, 1]) < 0.03


def _single_spin_samples(orc, w, n_steps):
    s = orc.System(w)
    S = w.S0.copy()
    s.mc(S, 0, 2000, record=False)
    m, _, _ = s.mc(S, 2000, n_steps)
    return m[:, 2]


@pytest.mark.parametrize("xi", [1.0, 3.0, 10.0])
def test_mc_boltzmann_uniaxial(orc, xi):
    ku = 1e-23
    w = single_spin(mu_s=1.5 * MU_B, k_u=ku, temperature=ku / (KB * xi), S0=(0, 0, 1), seed=21)
    cz = _single_spin_samples(orc, w, 400_000)
    mean, se = orc.block_stats(cz ** 2, 40)
    num = integrate.quad(lambda t: np.cos(t) ** 2 * np.sin(t) * np.exp(xi * np.cos(t) ** 2), 0, np.pi)[0]
    den = integrate.quad(lambda t: np.sin(t) * np.exp(xi * np.cos(t) ** 2), 0, np.pi)[0]
    assert abs(mean - num / den) < 4 * se + 2e-3, (mean, se, num / den)


@pytest.mark.parametrize("x", [0.5, 2.0, 5.0])
def test_mc_langevin_function_in_a_field(orc, x):
    """No anisotropy, field along +z: <cos theta> = coth(x) - 1/x with
    x = mu_s H / (kB T)."""
    mu, T = 1.5 * MU_B, 50.0
    H = x * KB * T / mu
    w = single_spin(mu_s=mu, k_u=0.0, H=(0.0, 0.0, H), temperature=T, S0=(1, 0, 0), seed=22)
    cz = _single_spin_samples(orc, w, 400_000)
    mean, se = orc.block_stats(cz, 40)
    assert abs(mean - (1.0 / np.tanh(x) - 1.0 / x)) < 4 * se + 2e-3, (mean, se)


def test_mc_at_zero_temperature_never_raises_the_energy(orc):
    w = sc_reference(L=6, temperature=0.0, seed=4)
    rng = np.random.default_rng(0)
    S = rng.standard_normal((w.n, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    s = orc.System(w)
    E0 = s.energy(S)
    _, E, acc = s.mc(S, 0, 50)
    assert E[0] <= E0 and np.all(np.diff(E) <= 1e-30)
    assert acc.sum() > 0 and E[-1] < E0


@pytest.mark.parametrize("T", [300.0, 400.0])
def test_mc_matches_paper_sc_magnetisation_fit(orc, T):
    """The paper fits its simple-cubic M(T) (J = 6.0e-21 J/link) with
    m = (1 - T/Tc)^beta, Tc = 631.82 K, beta = 0.334297."""
    w = sc_reference(L=12, temperature=T, seed=3)
    r, _ = orc.mc_average(orc.System(w), w.S0.copy(), 0, 1000, 3000, 10)
    fit = (1.0 - T / 631.82) ** 0.334297
    assert abs(r["m_abs"] - fit) < 0.03, (r["m_abs"], fit)
    assert 0.1 < r["acceptance"] < 0.9


def test_mc_agrees_with_llg_at_equilibrium(orc):
    """Monte Carlo and Langevin dynamics sample the same equilibrium
    (the paper's Monte Carlo vs LLG comparison)."""
    T = 400.0
    w = sc_reference(L=8, temperature=T, seed=6)
    w.alpha = 1.0
    mc, _ = orc.mc_average(orc.System(w), w.S0.copy(), 0, 2000, 20000, 20)
    llg, _ = orc.average(orc.System(w), w.S0.copy(), 0, 20000, 200000, 20)
    tol = 4 * np.hypot(mc["m_abs_se"], llg["m_abs_se"]) + 5e-3
    assert abs(mc["m_abs"] - llg["m_abs"]) < tol, (mc, llg)


def _chain_average(args):
    import oracle
    T, order, seed = args
    w = sc_reference(L=12, temperature=T, seed=seed)
    r, _ = oracle.mc_average(oracle.System(w), w.S0.copy(), 0, 2000, 4000, 10, order=order)
    return r["m_abs"], r["E"], r["acceptance"]


def test_random_site_order_matches_colour_sweeps():
    """The paper's Monte Carlo step is N trials on sites drawn at random;
    the GPU sweeps colour classes instead.  Both chains keep the Boltzmann
    distribution, so <|m|> and <E> of the sc 12^3 test system (J = 6e-21
    J/link) agree at 300 K and around Tc (600, 625, 650 K).  Errors come
    from eight independent chains per order (2000 equilibration + 4000
    averaging steps each): near Tc the correlation time is long, and the
    spread of independent chains measures it where blocks of one chain
    would not.  Bound: 3 standard errors of the difference."""
    temps = (300.0, 600.0, 625.0, 650.0)
    K = 8
    jobs = [(T, order, 1 + 100 * k + (0 if order == "random" else 50))
            for T in temps for order in ("random", "colour") for k in range(K)]
    with get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        out = np.array(pool.map(_chain_average, jobs)).reshape(len(temps), 2, K, 3)
    for t, T in enumerate(temps):
        for col, name in ((0, "<|m|>"), (1, "<E>")):
            x = out[t, :, :, col]
            mean = x.mean(axis=1)
            se = x.std(axis=1, ddof=1) / np.sqrt(K)
            diff = abs(mean[0] - mean[1])
            print(f"T = {T:.0f} K {name}: random {mean[0]:.5g} +- {se[0]:.2g}, colour {mean[1]:.5g} +- "
                  f"{se[1]:.2g}, |diff| / se {diff / np.hypot(*se):.2f}")
            assert diff <= 3 * np.hypot(*se), (T, name, mean, se)
        acc = out[t, :, :, 2].mean(axis=1)
        assert abs(acc[0] - acc[1]) < 0.01


def test_lattice_visit_order_and_its_colouring(orc):
    """The colouring's lattice visiting order groups the sites by basis site
    and by the parity of the cell's x + y + z (checked here from the site
    positions the lattice builder placed, not from the index arithmetic),
    and its greedy colouring is proper.  On the periodic bcc lattice with
    first and second neighbours it gives four classes of N/4 (the two
    sublattices, each split by parity: second neighbours join cells of
    opposite parity on one sublattice), where ascending order gives nine or
    ten unequal ones; on simple cubic it gives the two parity classes,
    the same as ascending order.  On an odd periodic edge the parity split
    is no colouring, and greedy still gives a proper one."""
    w = bcc((8, 8, 8), (True, True, True), second_neighbours=True)
    wb = bcc_block(cells=8)
    sysb = orc.System(wb)
    visit = sysb.lattice_visit()
    assert np.array_equal(np.sort(visit), np.arange(wb.n))
    pos = np.asarray(w.pos)
    b = (np.abs(pos[:, 0] - np.round(pos[:, 0])) > 0.25).astype(int)
    parity = np.floor(pos + 1e-9).astype(int).sum(axis=1) & 1
    key = 2 * b + parity
    assert np.all(np.diff(key[visit]) >= 0), "visit not grouped by (basis site, parity)"
    for g in range(4):   # ascending within a group
        grp = visit[key[visit] == g]
        assert np.all(np.diff(grp) > 0)
    rows = np.repeat(np.arange(wb.n), np.diff(sysb.row_ptr))
    c_lat = sysb.colours("lattice")
    c_asc = sysb.colours()
    for c in (c_lat, c_asc):
        assert np.all(c[rows] != c[sysb.col]), "a link joins two sites of one colour"
    assert np.array_equal(np.bincount(c_lat), [wb.n // 4] * 4)
    assert np.array_equal(c_lat, 2 * b + parity)
    assert c_asc.max() + 1 >= 9
    assert np.array_equal(c_asc, orc.greedy_colours(sysb.row_ptr, sysb.col)[0])
    ws = sc_reference(L=12)
    syss = orc.System(ws)
    assert np.array_equal(syss.colours("lattice"), syss.colours())
    assert syss.colours().max() == 1
    wo = bcc_block(cells=5)
    syso = orc.System(wo)
    c = syso.colours("lattice")
    rows = np.repeat(np.arange(wo.n), np.diff(syso.row_ptr))
    assert np.all(c[rows] != c[syso.col])
    assert c.max() + 1 > 4


def _bcc_chain_average(args):
    import oracle
    T, order, seed = args
    w = bcc_block(cells=6, temperature=T, seed=seed)
    r, _ = oracle.mc_average(oracle.System(w), w.S0.copy(), 0, 4000, 8000, 10, order=order,
                             visit="lattice" if order == "colour" else None)
    return r["m_abs"], r["E"], r["acceptance"]


def test_random_site_order_matches_lattice_ordered_colour_sweeps():
    """The four balanced colour classes of the lattice visiting order sample
    the paper's equilibrium too: on the bcc J1+J2 test block (6^3 cells, 432
    spins) <|m|> and <E> of the colour-class chain agree with the random-site
    chain at 800 K and near the block's ordering temperature (1300 K; mean
    field puts Tc near 1400 K).  Sixteen independent chains per order,
    4000 + 8000 steps each; bound 3 standard errors of the difference."""
    temps = (800.0, 1300.0)
    K = 16
    jobs = [(T, order, 11 + 100 * k + (0 if order == "random" else 50))
            for T in temps for order in ("random", "colour") for k in range(K)]
    with get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        out = np.array(pool.map(_bcc_chain_average, jobs)).reshape(len(temps), 2, K, 3)
    for t, T in enumerate(temps):
        for col, name in ((0, "<|m|>"), (1, "<E>")):
            x = out[t, :, :, col]
            mean = x.mean(axis=1)
            se = x.std(axis=1, ddof=1) / np.sqrt(K)
            diff = abs(mean[0] - mean[1])
            print(f"bcc T = {T:.0f} K {name}: random {mean[0]:.5g} +- {se[0]:.2g}, lattice-ordered colour "
                  f"{mean[1]:.5g} +- {se[1]:.2g}, |diff| / se {diff / np.hypot(*se):.2f}")
            assert diff <= 3 * np.hypot(*se), (T, name, mean, se)
        acc = out[t, :, :, 2].mean(axis=1)
        assert abs(acc[0] - acc[1]) < 0.01
