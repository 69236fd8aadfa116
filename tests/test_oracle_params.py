"""Closed-form pins for the oracle's strategy parameters.

The paper prints no parameter formula (Sec. 4.1 defers to the reference
code's defaults); the reading is the CMA-ES tutorial parameter set.  What is
fixed independently of that reading: the default population sizes of the
workloads (10/17/19/24/26 for n = 10/100/200/1000/2000), weights that are
positive, non-increasing and sum to one (Sec. 2.1, eq. (2)), mu_eff as the
variance-effective selection mass, and chi_n approximating E||N(0, I)||.
"""

import math

import numpy as np
import pytest
from scipy.special import gammaln

import oracle as O


@pytest.mark.parametrize("n,lam", [(1, 4), (2, 6), (10, 10), (100, 17), (200, 19), (1000, 24),
                                   (2000, 26)])
def test_default_lambda(n, lam):
    assert O.default_lambda(n) == lam


@pytest.mark.parametrize("n,lam", [(10, 10), (100, 17), (100, 8704), (1000, 24), (1000, 6144),
                                   (200, 19), (200, 9728), (2000, 4096), (3, 2), (5, 3)])
def test_weights_and_rates(n, lam):
    p = O.params(n, lam)
    assert p.mu == lam // 2 and p.w.shape == (p.mu,)
    assert abs(p.w.sum() - 1.0) < 1e-14
    assert np.all(p.w > 0) and np.all(np.diff(p.w) <= 0)
    # mu_eff = (sum w)^2 / sum w^2 for the unnormalised log weights as well
    wp = np.log((lam + 1) / 2.0) - np.log(np.arange(1, p.mu + 1))
    assert abs(p.mueff - wp.sum() ** 2 / np.sum(wp ** 2)) < 1e-10 * p.mueff
    assert 1.0 <= p.mueff <= p.mu + 1e-12
    for r in (p.cs, p.cc, p.c1):
        assert 0.0 < r <= 1.0
    assert 0.0 <= p.cmu < 1.0     # mu_eff = 1 gives cmu = 0 (rank-mu term off)
    assert p.c1 + p.cmu <= 1.0 + 1e-15
    assert p.ds >= 1.0 + p.cs - 1e-15
    assert p.kappa >= 1


@pytest.mark.parametrize("n", [1, 2, 5, 10, 40, 100, 200, 1000, 2000])
def test_chi_n_against_exact_expectation(n):
    exact = math.sqrt(2.0) * math.exp(gammaln((n + 1) / 2.0) - gammaln(n / 2.0))
    p = O.params(n, max(O.default_lambda(n), 2))
    assert abs(p.chin - exact) / exact < 1e-3


def test_chi_n_monte_carlo():
    n = 30
    z = np.random.default_rng(0).standard_normal((200000, n))
    emp = np.linalg.norm(z, axis=1).mean()
    assert abs(O.params(n, 12).chin - emp) / emp < 2e-3


def test_equal_weights_limit():
    # lambda = 2 -> mu = 1, single weight 1, mu_eff = 1
    p = O.params(5, 2)
    assert p.mu == 1 and p.w[0] == 1.0 and p.mueff == 1.0


def test_eigen_interval_reading():
    # ceil(1/(10 n (c1 + cmu))), at least one generation
    for n, lam in [(10, 10), (100, 17), (1000, 24), (1000, 6144), (2000, 4096), (200, 19)]:
        p = O.params(n, lam)
        assert p.kappa == max(1, math.ceil(1.0 / (10 * n * (p.c1 + p.cmu))))
    assert O.params(1000, 6144).kappa == 1 and O.params(2000, 4096).kappa == 1
    assert O.params(10, 10, kappa=1).kappa == 1


def test_params_against_independent_table():
    """Values evaluated independently of this code (tests/golden/params_table.json)."""
    import json
    import os
    tab = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "params_table.json")))
    tol = tab["rel_tol"]
    for row in tab["rows"]:
        p = O.params(row["n"], row["lam"])
        assert p.mu == row["mu"]
        for k in ("mueff", "cs", "ds", "cc", "c1", "cmu", "chin"):
            want = row[k]
            digits = len(str(want).replace("-", "").replace(".", "").split("e")[0].lstrip("0"))
            rt = max(tol, 0.6 * 10.0 ** (1 - digits))
            assert abs(getattr(p, k) - want) <= rt * abs(want), (row["n"], row["lam"], k)
    np.testing.assert_allclose(O.params(10, 10).w, tab["weights_n10_lam10"], rtol=0, atol=6e-7)
