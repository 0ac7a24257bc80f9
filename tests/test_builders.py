"""The C ABI's structure builders (sllg_build_sc / _bcc / _fcc_sphere; host
only, no GPU): the same CSR lists, types and positions as the seeded input
generators of the tests (spin_systems.lattice), which the oracle's
lattice tests pin against brute force; the two-call protocol and its errors;
and a built block declared cell by cell qualifies for the fused step."""
import ctypes

import numpy as np
import pytest

import paper_1310_6143_amd as sl
from spin_systems.lattice import bcc, fcc_sphere, simple_cubic


def _same(built, lat):
    row_ptr, col, typ, pos = built
    assert np.array_equal(row_ptr, lat.row_ptr)
    assert np.array_equal(col, lat.col)
    assert np.array_equal(typ, lat.ntype)
    assert np.array_equal(pos, lat.pos)


@pytest.mark.parametrize("dims,periodic", [((3, 3, 3), (1, 1, 1)), ((5, 4, 7), (1, 1, 1)), ((6, 5, 4), (1, 1, 0)),
                                           ((4, 1, 3), (1, 0, 1)), ((2, 2, 2), (0, 0, 0))])
def test_sc_matches_generator(dims, periodic):
    _same(sl.build_sc(dims, periodic), simple_cubic(dims, tuple(bool(p) for p in periodic)))


@pytest.mark.parametrize("second", [False, True])
@pytest.mark.parametrize("dims,periodic", [((3, 3, 3), (1, 1, 1)), ((6, 5, 4), (1, 1, 1)), ((8, 7, 5), (1, 1, 0)),
                                           ((2, 3, 1), (0, 1, 0))])
def test_bcc_matches_generator(dims, periodic, second):
    _same(sl.build_bcc(dims, periodic, second), bcc(dims, tuple(bool(p) for p in periodic), second_neighbours=second))


@pytest.mark.parametrize("a_nm,radius_nm", [(0.3524, 0.0), (0.3524, 0.5), (0.3524, 1.5), (0.3524, 2.2), (0.4, 1.0)])
def test_fcc_sphere_matches_generator(a_nm, radius_nm):
    _same(sl.build_fcc_sphere(a_nm, radius_nm), fcc_sphere(a_nm, radius_nm))


def test_fcc_sphere_shells():
    """Every bulk site has 12 links at a / sqrt(2); the particle is a ball."""
    row_ptr, col, _, pos = sl.build_fcc_sphere(0.3524, 2.0)
    deg = np.diff(row_ptr)
    assert deg.max() == 12 and deg.min() >= 3
    i = np.repeat(np.arange(deg.size), deg)
    d = np.linalg.norm(pos[i] - pos[col], axis=1)
    assert np.allclose(d, np.sqrt(0.5))
    r = np.linalg.norm(pos, axis=1) * 0.3524
    assert r.max() <= 2.0 + 1e-9
    assert np.all(deg[r < 2.0 - 0.3524] == 12)


def test_protocol_and_errors():
    L = sl.lib()
    cells = np.array([4, 4, 4], dtype=np.int32)
    per = np.array([1, 1, 1], dtype=np.int32)
    n, nnz = ctypes.c_int64(0), ctypes.c_int64(0)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert L.sllg_build_sc(P(cells), P(per), ctypes.byref(n), ctypes.byref(nnz), None, None, None, None) == 0
    assert (n.value, nnz.value) == (64, 384)
    rp = np.empty(65, dtype=np.int64)
    col = np.empty(384, dtype=np.int32)
    bad = ctypes.c_int64(383)
    # counts that differ from the first call's
    assert L.sllg_build_sc(P(cells), P(per), ctypes.byref(n), ctypes.byref(bad), P(rp), P(col), None, None) == -1
    assert b"counts" in L.sllg_last_error(None)
    # row_ptr without col
    assert L.sllg_build_sc(P(cells), P(per), ctypes.byref(n), ctypes.byref(nnz), P(rp), None, None, None) == -1
    # type and pos are optional
    assert L.sllg_build_sc(P(cells), P(per), ctypes.byref(n), ctypes.byref(nnz), P(rp), P(col), None, None) == 0
    assert np.array_equal(col, simple_cubic((4, 4, 4)).col)
    # NULL counts
    assert L.sllg_build_sc(P(cells), P(per), None, ctypes.byref(nnz), None, None, None, None) == -1
    # a periodic axis of 2 cells, no cells, too many sites, bad sphere
    for c, p in (((2, 4, 4), (1, 1, 1)), ((0, 4, 4), (0, 0, 0)), ((1024, 1024, 512), (1, 1, 1))):
        with pytest.raises(sl.SllgError):
            sl.build_sc(c, p)
    with pytest.raises(sl.SllgError):
        sl.build_bcc((2, 3, 3), (1, 1, 1))
    for a, r in ((0.0, 1.0), (0.35, -1.0), (float("nan"), 1.0), (0.35, 1e6)):
        with pytest.raises(sl.SllgError):
            sl.build_fcc_sphere(a, r)


def test_built_block_takes_the_fused_step():
    """The builders number sites as sllg_set_lattice declares them: a bcc
    block built here, declared cell by cell, qualifies for the fused step
    (checked on the host; the device is not opened)."""
    row_ptr, col, typ, _ = sl.build_bcc((8, 8, 8), (1, 1, 1), second_neighbours=True)
    n = row_ptr.size - 1
    s = sl.SpinSystem(n, sl.FP32)
    try:
        s.set_neighbours(row_ptr, col, typ, [7.05e-21, 3.0e-21])
        s.set_lattice(2, (8, 8, 8), (1, 1, 1))
        assert s.get_option("lattice") == 2
    finally:
        s.close()
