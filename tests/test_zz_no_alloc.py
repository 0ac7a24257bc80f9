"""The entry point that allocates no device memory,
sllg_thermal_normals_noalloc, against sllg_thermal_normals (which
allocates its staging buffer per call), through the C ABI: the same normals
bit for bit, on two calls in a row, the second smaller, in both
precisions; sizes beyond its fixed scratch are refused."""
import numpy as np
import pytest

import paper_1310_6143_amd as sl

pytestmark = pytest.mark.gpu

MAX_SITES = 1 << 18


@pytest.mark.parametrize("precision", [sl.FP64, sl.FP32])
def test_noalloc_normals_match_allocating_entry_point(precision):
    for seed, step, n in ((42, 7, MAX_SITES), (9, (1 << 32) + 3, 1000)):
        got = sl.thermal_normals_noalloc(seed, step, n, precision)
        ref = sl.thermal_normals(seed, step, n, precision)
        assert got.shape == (n, 3)
        assert np.array_equal(got, ref), (seed, step, n)
    # the smaller call left the rest of the scratch as it was; a third call
    # with other inputs still returns its own values
    got = sl.thermal_normals_noalloc(5, 0, 17, precision)
    assert np.array_equal(got, sl.thermal_normals(5, 0, 17, precision))


def test_noalloc_refuses_sizes_beyond_its_scratch():
    for n in (0, MAX_SITES + 1):
        with pytest.raises(sl.SllgError) as e:
            sl.thermal_normals_noalloc(1, 0, n)
        assert e.value.name == "SLLG_E_ARG"
    with pytest.raises(sl.SllgError) as e:
        sl.thermal_normals_noalloc(1, 0, MAX_SITES + 1)
    assert "scratch" in str(e.value)
