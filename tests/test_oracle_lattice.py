"""Pins for the neighbour lists (inputs to both sides) and for the exchange
convention of the oracle.

- The CSR builders in ``spin_systems`` are compared, as sets per row, with
  the oracle's brute-force all-pairs search on small crystals.
- Coordination numbers: sc 6, bcc 8 (+6 second neighbours), fcc 12, as in
  Table 2 and the sc test system of the Monte Carlo section.
- The mean-field relation between J and Tc (section "Exchange energy",
  J = 3 kB Tc / (eps z)) is checked against Table 2, and the oracle's
  exchange field at full alignment reproduces the Table 2 Curie
  temperatures: this fixes "J per link" (each link counted once).
"""
import json
import os

import numpy as np
import pytest

from spin_systems import bcc, fcc_sphere, sc_long_range, simple_cubic, MU_B
from spin_systems import sc_reference, bcc_film, fcc_nanoparticle, bcc_block

HERE = os.path.dirname(os.path.abspath(__file__))
TABLES = json.load(open(os.path.join(HERE, "golden", "paper_tables.json")))


def _rows_as_sets(row_ptr, col, ntype):
    return [set(zip(col[row_ptr[i]:row_ptr[i + 1]].tolist(), ntype[row_ptr[i]:row_ptr[i + 1]].tolist()))
            for i in range(row_ptr.size - 1)]


def _check_against_bruteforce(orc, lat, box, shells, max_degree=64):
    rp, c, t = orc.neighbours(lat.pos, box, shells, max_degree)
    ours = _rows_as_sets(lat.row_ptr, lat.col, lat.ntype)
    ref = _rows_as_sets(rp, c, t)
    assert ours == ref
    # ascending columns within each row
    for i in range(lat.n):
        row = lat.col[lat.row_ptr[i]:lat.row_ptr[i + 1]]
        assert np.all(np.diff(row) > 0)


def test_sc_periodic_matches_bruteforce(orc):
    lat = simple_cubic((5, 4, 3), (True, True, True))
    _check_against_bruteforce(orc, lat, [5, 4, 3], [(0.99, 1.01)])
    assert np.all(lat.degree() == 6)


def test_long_range_sc_matches_bruteforce(orc):
    """Every pair within r_cut, 16 radial bins of equal width as types: the
    count of integer vectors of length <= 3.2 is 146."""
    lat = sc_long_range(7, 3.2)
    # the builder's bins are closed on the left; the brute force takes the
    # first bin whose closed interval holds r: nudge the inner bounds apart
    shells = [(lo + 1e-9 if t > 0 else lo - 1e-9, hi - 1e-9 if t < 15 else hi + 1e-9)
              for t, (lo, hi) in enumerate(lat.shells)]
    _check_against_bruteforce(orc, lat, [7, 7, 7], shells, max_degree=200)
    assert np.all(lat.degree() == 146)


def test_sc_open_matches_bruteforce(orc):
    lat = simple_cubic((4, 3, 5), (False, True, False))
    _check_against_bruteforce(orc, lat, [0, 3, 0], [(0.99, 1.01)])


def test_bcc_with_second_neighbours_matches_bruteforce(orc):
    lat = bcc((4, 3, 5), (True, True, True), second_neighbours=True)
    d1 = np.sqrt(3) / 2
    _check_against_bruteforce(orc, lat, [4, 3, 5], [(d1 - 0.01, d1 + 0.01), (0.99, 1.01)])
    assert np.all(lat.degree() == 14)
    assert np.all(np.bincount(lat.ntype) == [8 * lat.n, 6 * lat.n])


def test_bcc_film_matches_bruteforce(orc):
    lat = bcc((4, 4, 3), (True, True, False))
    d1 = np.sqrt(3) / 2
    _check_against_bruteforce(orc, lat, [4, 4, 0], [(d1 - 0.01, d1 + 0.01)])
    deg = lat.degree()
    z = lat.pos[:, 2]
    assert np.all(deg[(z == 0.0)] == 4)          # bottom corner sites
    assert np.all(deg[(z == 2.5)] == 4)          # top body-centre sites
    assert np.all(deg[(z > 0.0) & (z < 2.5)] == 8)


def test_fcc_sphere_matches_bruteforce(orc):
    lat = fcc_sphere(0.3524, 0.9)
    _check_against_bruteforce(orc, lat, [0, 0, 0], [(1 / np.sqrt(2) - 0.01, 1 / np.sqrt(2) + 0.01)])
    assert lat.degree().max() == 12
    # the centre site is fully coordinated
    centre = np.argmin(np.linalg.norm(lat.pos, axis=1))
    assert lat.degree()[centre] == 12


def _symmetric(lat):
    rows = np.repeat(np.arange(lat.n), lat.degree())
    fwd = set(zip(rows.tolist(), lat.col.tolist(), lat.ntype.tolist()))
    bwd = set(zip(lat.col.tolist(), rows.tolist(), lat.ntype.tolist()))
    return fwd == bwd


def test_config_sizes_and_symmetry():
    w0 = sc_reference()
    assert (w0.n, w0.lattice.nnz) == (4096, 24576)
    assert _symmetric(w0.lattice)
    w1 = bcc_film()
    assert (w1.n, w1.lattice.nnz) == (131072, 1015808)
    assert np.bincount(w1.lattice.degree()).tolist()[4] == 2 * 64 * 64
    w2 = fcc_nanoparticle()
    assert (w2.n, w2.lattice.nnz) == (196053, 2297664)
    assert _symmetric(w2.lattice)
    assert int((w2.lattice.degree() < 12).sum()) == 16292
    w4 = bcc_block(32)
    assert (w4.n, w4.lattice.nnz) == (65536, 65536 * 14)
    assert _symmetric(w4.lattice)


def test_table2_exchange_reproduces_tc():
    kb = TABLES["table1"]["k_B"]
    for name, el in TABLES["table2"].items():
        tc = el["J"] * el["eps"] * el["z"] / (3 * kb)
        assert abs(tc - el["Tc"]) < 0.6, (name, tc)


def test_oracle_exchange_field_gives_table2_tc(orc):
    """At full alignment the oracle's exchange field on a bulk site is
    z J / mu_s; the mean-field Curie temperature mu_s |H| / (3 kB), scaled by
    Table 2's spin-wave factor eps, must give Table 2's Tc.  A double-counted
    link (factor 2) would miss by 100%."""
    kb = TABLES["table1"]["k_B"]
    assert orc.KB == kb
    for name, lat in (("Fe", bcc((4, 4, 4))), ("Ni", fcc_sphere(0.3524, 0.6))):
        el = TABLES["table2"][name]
        n = lat.n
        mu = el["mu_s_muB"] * MU_B

        class W:
            pass
        w = W()
        w.lattice, w.J = lat, np.array([el["J"]])
        w.mu_s, w.k_u, w.easy_axis = np.full(n, mu), np.zeros(n), np.tile([0, 0, 1.0], (n, 1))
        w.alpha, w.gamma, w.dt, w.temperature, w.H, w.seed = 0.1, 1.76e11, 1e-16, 0.0, np.zeros(3), 0
        s = orc.System(w)
        S = np.tile([0.0, 0.0, 1.0], (n, 1))
        h = s.fields(S)
        bulk = int(np.argmax(lat.degree()))
        assert lat.degree()[bulk] == el["z"]
        tc = el["eps"] * mu * np.linalg.norm(h[bulk]) / (3 * kb)
        assert abs(tc - el["Tc"]) < 0.6, (name, tc)


@pytest.mark.slow
def test_large_bcc_block_shape():
    w = bcc_block(160)
    assert (w.n, w.lattice.nnz) == (8_192_000, 114_688_000)
    assert np.all(w.lattice.degree() == 14)
