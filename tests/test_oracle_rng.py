"""Pins for the oracle's counter-based noise (Philox4x32-10 + Box-Muller).

The paper only asks for three independent standard normals per spin per
step ("Langevin Dynamics"); which generator makes them is free.  The oracle
uses Philox4x32-10, pinned here to (1) the published known-answer values,
(2) rocRAND's independent implementation of the same generator, and
(3) the standard normal distribution (scipy) for the Box-Muller output.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    for ctr, key, expect in _kat():
        out = orc.philox4x32_10([ctr], [key])[0]
        assert [int(x) for x in out] == expect


@pytest.fixture(scope="module")
def rocrand_dump(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("g++ or rocRAND headers not available")
    exe = tmp_path_factory.mktemp("rr") / "philox_dump"
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "helpers", "rocrand_philox_dump.cpp"), "-o", str(exe)],
                   check=True)
    return str(exe)


def test_philox_matches_rocrand(orc, rocrand_dump):
    rng = np.random.default_rng(7)
    m = 20000
    ctr = rng.integers(0, 2**32, size=(m, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(m, 2), dtype=np.uint64).astype(np.uint32)
    # include the counter layout the dynamics uses: (site, step lo, step hi, purpose)
    ctr[:100, 0] = np.arange(100)
    ctr[:100, 1] = 12345
    ctr[:100, 2] = 0
    ctr[:100, 3] = 0
    text = "\n".join(" ".join(f"{int(v):08x}" for v in np.concatenate([c, k]))
                     for c, k in zip(ctr, key))
    res = subprocess.run([rocrand_dump], input=text, capture_output=True, text=True, check=True)
    lib_out = np.array([[int(t, 16) for t in line.split()] for line in res.stdout.split("\n") if line],
                       dtype=np.uint64)
    ours = orc.philox4x32_10(ctr, key).astype(np.uint64)
    assert lib_out.shape == ours.shape
    assert np.array_equal(lib_out, ours)


def test_gaussians_are_standard_normal(orc):
    # 40 steps x 5000 sites = 200k triples
    g = np.concatenate([orc.gaussians(42, step, np.arange(5000)) for step in range(40)])
    for c in range(3):
        x = g[:, c]
        ks = stats.kstest(x, "norm")
        assert ks.pvalue > 1e-3, (c, ks)
        se = 1.0 / np.sqrt(x.size)
        assert abs(x.mean()) < 5 * se
        assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0) * se
        assert abs(stats.kurtosis(x, fisher=False) - 3.0) < 5 * np.sqrt(24.0) * se
    corr = np.corrcoef(g.T)
    assert np.all(np.abs(corr - np.eye(3)) < 5 / np.sqrt(g.shape[0]))


def test_gaussians_depend_on_every_counter_word(orc):
    base = orc.gaussians(42, 7, [3])[0]
    assert not np.allclose(base, orc.gaussians(43, 7, [3])[0])           # key
    assert not np.allclose(base, orc.gaussians(42, 8, [3])[0])           # step low word
    assert not np.allclose(base, orc.gaussians(42, 7 + (1 << 32), [3])[0])  # step high word
    assert not np.allclose(base, orc.gaussians(42, 7, [4])[0])           # site
    assert not np.allclose(base, orc.gaussians(42, 7, [3], purpose=1)[0])  # purpose word
    assert np.array_equal(base, orc.gaussians(42, 7, [3])[0])            # pure function


def test_box_muller_uses_the_documented_words(orc):
    """The first normal must be sqrt(-2 ln((r0+1)/2^32)) cos(2 pi r1/2^32) of
    the Philox block at counter (site, step lo, step hi, 0): this fixes the
    counter layout the GPU side has to reproduce."""
    seed, step, site = 0x1234567890ABCDEF, (5 << 32) + 17, 99
    r = orc.philox4x32_10([[site, step & 0xFFFFFFFF, step >> 32, 0]],
                          [[seed & 0xFFFFFFFF, seed >> 32]])[0].astype(np.float64)
    g = orc.gaussians(seed, step, [site])[0]
    u1 = (r[0] + 1.0) / 2**32
    u2 = r[1] / 2**32
    u3 = (r[2] + 1.0) / 2**32
    u4 = r[3] / 2**32
    expect = [np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2),
              np.sqrt(-2 * np.log(u1)) * np.sin(2 * np.pi * u2),
              np.sqrt(-2 * np.log(u3)) * np.cos(2 * np.pi * u4)]
    assert np.allclose(g, expect, rtol=1e-13, atol=1e-13)
