"""Pins for the oracle's random numbers (z_k ~ N(0, I) of eq. (1)).

* Philox4x32-10 raw blocks equal rocRAND's header-only engine, built on the
  host from tests/golden/philox_rocrand_ref.cpp.
* Box-Muller normals have N(0,1) moments and pass a Kolmogorov-Smirnov test.
* The initial mean is uniform in the search box (Sec. 4.1).
"""

import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _build_ref(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    inc = "/opt/rocm/include"
    if cxx is None or not os.path.isdir(os.path.join(inc, "rocrand")):
        pytest.skip("no host C++ compiler or rocRAND headers")
    out = tmp_path_factory.mktemp("philox") / "philox_ref"
    src = os.path.join(HERE, "golden", "philox_rocrand_ref.cpp")
    subprocess.run([cxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I", inc, src, "-o", str(out)],
                   check=True, capture_output=True)
    return str(out)


@pytest.fixture(scope="module")
def philox_ref(tmp_path_factory):
    return _build_ref(tmp_path_factory)


def test_philox_matches_rocrand(philox_ref):
    rng = np.random.default_rng(12345)
    rows = [(0, 0, 0, 0, 0, 0),
            (0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF),
            (1, 2, 3, 4, 5, 6)]
    for _ in range(200):
        c = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        k = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        c[1] %= 2 ** 30
        rows.append(tuple(int(v) for v in (*c, *k)))
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    res = subprocess.run([philox_ref], input=inp, capture_output=True, text=True, check=True)
    want = np.array([[int(t) for t in line.split()] for line in res.stdout.strip().splitlines()],
                    dtype=np.uint64)
    arr = np.array(rows, dtype=np.uint64)
    got = O.philox4x32_10(arr[:, 0], arr[:, 1], arr[:, 2], arr[:, 3], arr[:, 4], arr[:, 5])
    got = np.stack([g.astype(np.uint64) for g in got], axis=1)
    assert want.shape == got.shape
    np.testing.assert_array_equal(got, want)


def test_unit_map_open_interval():
    u = O.u32_to_unit(np.array([0, 1, 2 ** 31, 2 ** 32 - 1], dtype=np.uint64))
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert u[2] == 0.5 + 0.5 / 2 ** 32


def test_normals_moments_and_ks():
    Z = O.normals(seed=7, restart=0, gen=0, n=101, lam=4000)   # ragged n (not /4)
    z = Z.ravel()
    assert Z.shape == (101, 4000)
    assert abs(z.mean()) < 5.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 8.0 * np.sqrt(2.0 / z.size)
    assert abs(stats.skew(z)) < 0.02 and abs(stats.kurtosis(z)) < 0.04
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # pairs from one Box-Muller draw are uncorrelated
    assert abs(np.corrcoef(Z[0], Z[1])[0, 1]) < 5.0 / np.sqrt(4000)


def test_normals_counter_structure():
    a = O.normals(3, 1, 5, 10, 7)
    b = O.normals(3, 1, 5, 12, 9)
    np.testing.assert_array_equal(a, b[:10, :7])      # prefix property in n and lambda
    assert not np.allclose(a, O.normals(3, 1, 6, 10, 7))   # generation word matters
    assert not np.allclose(a, O.normals(3, 2, 5, 10, 7))   # restart word matters
    assert not np.allclose(a, O.normals(4, 1, 5, 10, 7))   # key matters
    assert not np.allclose(O.normals(1 << 32, 0, 0, 4, 4), O.normals(0, 0, 0, 4, 4))


def test_init_mean_uniform_in_box():
    m = O.init_mean(seed=11, restart=0, n=20000, lo=-4.0, hi=4.0)
    assert m.min() > -4.0 and m.max() < 4.0
    assert stats.kstest((m + 4.0) / 8.0, "uniform").pvalue > 1e-3
    assert not np.allclose(m[:10], O.init_mean(11, 1, 10, -4.0, 4.0))
