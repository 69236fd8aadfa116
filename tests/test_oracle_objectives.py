"""Pins of the oracle's synthetic objectives (the stand-ins for the benchmark
functions of the paper's Sec. 4.1) against closed forms that do not retype
their formulas:

* every objective is 0 at its optimum x*, whatever the rotation R;
* the rotated ellipsoid along the rotated axis R^T e_i (x = x* + t R^T e_i)
  equals t^2 10^(6 (i-1)/(n-1)): the axis scales run from 1 to 10^6
  (condition 1e6), in order;
* the rotated Rastrigin at integer u = R (x - x*) equals sum u_i^2 (the
  cosine term cancels the 10 n offset), and at u_i = 1/2 for all i it equals
  20.25 n (every cosine is -1);
* the sphere is the squared distance to x*;
* n = 1, where the ellipsoid exponent 6 (i-1)/(n-1) is undefined, reduces
  every objective to u^2 (plus the Rastrigin cosine term).

A wrong exponent, a dropped or doubled offset, R used where R^T belongs, or
x* added instead of subtracted fails at least one of these.
"""

import math

import numpy as np
import pytest

import oracle as O
import synth


def _point(R, xs, U):
    """x with R (x - x*) = U column by column (R orthogonal)."""
    return xs[:, None] + R.T @ U


@pytest.mark.parametrize("n", [1, 2, 7, 50])
def test_all_objectives_vanish_at_the_optimum(n):
    R, xs = synth.problem(n, seed=n + 11)
    X = np.repeat(xs[:, None], 3, axis=1)
    assert np.all(O.sphere(X, xs) == 0.0)
    assert np.max(np.abs(O.rot_ellipsoid(X, R, xs))) == 0.0
    assert np.max(np.abs(O.rot_rastrigin(X, R, xs))) < 1e-12 * n
    for kind in ("sphere", "ellipsoid", "rastrigin"):
        assert abs(O.Objective(kind, R, xs)(X)[0]) < 1e-12 * n, kind


@pytest.mark.parametrize("n", [2, 5, 100])
def test_rotated_ellipsoid_axis_scales(n):
    R, xs = synth.problem(n, seed=3 * n)
    t = 0.37
    U = t * np.eye(n)                      # column i: t e_i in rotated coordinates
    f = O.rot_ellipsoid(_point(R, xs, U), R, xs)
    expect = np.array([t * t * 10.0 ** (6.0 * i / (n - 1)) for i in range(n)])
    assert np.allclose(f, expect, rtol=1e-12, atol=0.0)
    assert f[0] == pytest.approx(t * t, rel=1e-12)
    assert f[-1] / f[0] == pytest.approx(1e6, rel=1e-12)      # condition number of the ellipsoid
    assert np.all(np.diff(f) > 0)


def test_rotated_ellipsoid_is_a_quadratic_form():
    """f(x* + s v) = s^2 f(x* + v) for any direction v."""
    n = 30
    R, xs = synth.problem(n, seed=4)
    v = synth.rng(9).standard_normal((n, 1))
    f1 = O.rot_ellipsoid(xs[:, None] + v, R, xs)[0]
    f3 = O.rot_ellipsoid(xs[:, None] + 3.0 * v, R, xs)[0]
    assert f3 == pytest.approx(9.0 * f1, rel=1e-12)


@pytest.mark.parametrize("n", [1, 3, 40])
def test_rotated_rastrigin_at_integer_and_half_points(n):
    R, xs = synth.problem(n, seed=n + 5)
    g = synth.rng(n)
    U = g.integers(-3, 4, size=(n, 6)).astype(np.float64)
    f = O.rot_rastrigin(_point(R, xs, U), R, xs)
    assert np.allclose(f, np.sum(U * U, axis=0), rtol=0.0, atol=1e-9 * n)
    half = np.full((n, 1), 0.5)
    fh = O.rot_rastrigin(_point(R, xs, half), R, xs)[0]
    assert fh == pytest.approx(20.25 * n, rel=1e-12)


def test_rastrigin_unrotated_matches_integer_closed_form():
    n = 12
    xs = synth.optimum(n, 2)
    U = synth.rng(1).integers(-2, 3, size=(n, 4)).astype(np.float64)
    f = O.rot_rastrigin(xs[:, None] + U, None, xs)
    assert np.allclose(f, np.sum(U * U, axis=0), atol=1e-10)
    assert O.rot_rastrigin(np.zeros((n, 1)))[0] == 0.0      # no shift, no rotation: optimum at the origin


def test_sphere_is_squared_distance():
    n = 9
    xs = synth.optimum(n, 8)
    X = synth.rng(3).standard_normal((n, 5))
    d = np.array([math.dist(X[:, k], xs) ** 2 for k in range(5)])
    assert np.allclose(O.sphere(X, xs), d, rtol=1e-13)
    R = synth.haar_rotation(n, 1)    # the sphere is rotation invariant
    assert np.allclose(O.Objective("sphere", R, xs)(X), d, rtol=1e-12)


def test_one_dimension_edge_case():
    xs = np.array([1.25])
    R = np.array([[-1.0]])
    u = np.array([[0.5, -2.0, 3.0]])
    X = xs[:, None] + R.T @ u
    assert np.allclose(O.rot_ellipsoid(X, R, xs), u[0] ** 2, rtol=1e-15)
    assert np.allclose(O.sphere(X, xs), u[0] ** 2, rtol=1e-15)
    expect = 10.0 + u[0] ** 2 - 10.0 * np.cos(2.0 * np.pi * u[0])
    assert np.allclose(O.rot_rastrigin(X, R, xs), expect, rtol=1e-14)
