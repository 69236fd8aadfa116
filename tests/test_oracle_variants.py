"""Pins of the oracle's CMA-ES variants (active negative weights; the
separable, large-scale variant), which the paper names as future work
(Sec. 5).  Each is tied to something other than its own formula: a positive
definiteness guarantee, an entry-by-entry form with an independent C^{-1/2},
special cases that reduce to the standard update, and convergence."""

import math

import numpy as np
import pytest

import oracle as O
import synth


@pytest.mark.parametrize("n,lam", [(10, 10), (10, 11), (40, 15), (200, 19), (5, 2), (1000, 24)])
def test_active_weights(n, lam):
    ps, pa = O.params(n, lam), O.params(n, lam, variant="active")
    mu = lam // 2
    assert np.array_equal(pa.w, ps.w) and pa.mueff == ps.mueff and pa.c1 == ps.c1 and pa.cmu == ps.cmu
    assert np.all(pa.w_all[:mu] > 0) and np.all(pa.w_all[mu:] <= 0)
    assert np.all(np.diff(pa.w_all) <= 0)                     # better rank, larger weight
    if lam % 2 == 1:
        assert pa.w_all[mu] == 0.0                            # ln((lam+1)/2) - ln(mu+1) = 0
    neg = -pa.w_all[mu:].sum()
    if pa.cmu == 0.0:                  # lam = 2: no rank-mu term, so no negative weights
        assert neg == 0.0 and pa.sumw == 1.0
        return
    assert 0.0 < neg <= 1.0 + pa.c1 / pa.cmu + 1e-12
    # the update cannot lose positive definiteness: cmu n sum|w^-| <= 1 - c1 - cmu
    assert pa.cmu * n * neg <= 1.0 - pa.c1 - pa.cmu + 1e-12
    assert pa.sumw == pytest.approx(1.0 - neg, rel=1e-14)


def _adversarial(n, lam, scale):
    """C = I, every negative-rank step along e_0 (of length `scale`), every
    positive-rank step and p_c orthogonal to it."""
    g = synth.rng(n + lam)
    Y = g.standard_normal((n, lam))
    Y[0, :] = 0.0
    order = np.arange(lam)
    Y[:, lam // 2:] = 0.0
    Y[0, lam // 2:] = scale
    pc = g.standard_normal(n)
    pc[0] = 0.0
    return Y, order, pc


@pytest.mark.parametrize("scale", [1e-3, 1.0, 1e3])
@pytest.mark.parametrize("n,lam", [(10, 10), (40, 100), (5, 64)])
def test_active_update_stays_positive_definite(n, lam, scale):
    p = O.params(n, lam, variant="active")
    Y, order, pc = _adversarial(n, lam, scale)
    C = O.covariance_update(np.eye(n), pc, Y, order, p, 1.0, np.eye(n), np.ones(n))
    assert np.linalg.eigvalsh(C)[0] > 0.0
    # without the n / ||C^{-1/2} y||^2 scaling long negative steps would break it
    q = O.params(n, lam, variant="active")
    q.w_all = q.w_all.copy()
    a = 1.0 - q.c1 - q.cmu * q.sumw
    Ys = Y[:, order]
    raw = a * np.eye(n) + q.c1 * np.outer(pc, pc) + q.cmu * ((Ys * q.w_all[None, :]) @ Ys.T)
    if scale >= 1e3:
        assert np.linalg.eigvalsh(raw)[0] < 0.0


def test_active_update_entry_by_entry():
    n, lam = 7, 12
    st = synth.random_state(n, lam, seed=3, cond=50.0)
    p = O.params(n, lam, variant="active")
    g = synth.rng(11)
    Y = st["B"] @ (st["D"][:, None] * g.standard_normal((n, lam)))
    order = g.permutation(lam)
    pc = st["p_c"]
    C = st["C"]
    got = O.covariance_update(C, pc, Y, order, p, 0.0, st["B"], st["D"])
    # C^{-1/2} from an eigendecomposition of C itself (not from B, D)
    ev, V = np.linalg.eigh(C)
    Cmh = V @ np.diag(ev ** -0.5) @ V.T
    hs = 0.0
    a = 1.0 - p.c1 - p.cmu * sum(p.w_all) + (1.0 - hs) * p.c1 * p.cc * (2.0 - p.cc)
    want = np.zeros((n, n))
    for j in range(n):
        for k in range(n):
            acc = 0.0
            for r in range(lam):
                y = Y[:, order[r]]
                wr = p.w_all[r]
                if wr < 0:
                    wr *= n / float(np.sum((Cmh @ y) ** 2))
                acc += wr * y[j] * y[k]
            want[j, k] = a * C[j, k] + p.c1 * pc[j] * pc[k] + p.cmu * acc
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_active_without_negative_weights_is_the_standard_update():
    n, lam = 12, 20
    st = synth.random_state(n, lam, seed=5)
    g = synth.rng(2)
    Y = g.standard_normal((n, lam))
    order = g.permutation(lam)
    ps_, pa = O.params(n, lam), O.params(n, lam, variant="active")
    pa.w_all = pa.w_all.copy()
    pa.w_all[lam // 2:] = 0.0
    pa.sumw = 1.0
    a = O.covariance_update(st["C"], st["p_c"], Y, order, pa, 1.0, st["B"], st["D"])
    b = O.covariance_update(st["C"], st["p_c"], Y, order, ps_, 1.0)
    assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(b))


def test_separable_rates_and_one_dimension():
    for n, lam in [(10, 10), (100, 17), (1000, 24)]:
        ps_, pv = O.params(n, lam), O.params(n, lam, variant="separable")
        assert pv.c1 == pytest.approx(min(1.0, ps_.c1 * (n + 2) / 3.0))
        assert pv.cmu == pytest.approx(min(1.0 - pv.c1, ps_.cmu * (n + 2) / 3.0))
        assert pv.kappa == 1
    # n = 1: (n + 2) / 3 = 1, so the separable variant is the standard one
    a = O.new_descent(1, 6, 1.0, 7, kappa=1)
    b = O.new_descent(1, 6, 1.0, 7, kappa=1, variant="separable")
    for _ in range(30):
        O.generation(a, O.Objective("sphere"))
        O.generation(b, O.Objective("sphere"))
    # equal up to the summation order of the rank-mu term
    assert a.m[0] == pytest.approx(b.m[0], rel=1e-10) and a.sigma == pytest.approx(b.sigma, rel=1e-10)
    assert a.C[0, 0] == pytest.approx(b.C[0, 0], rel=1e-10)


def test_separable_update_is_the_diagonal_of_the_standard_one():
    n, lam = 9, 16
    st = synth.random_state(n, lam, seed=8)
    Cd = np.diag(np.diag(st["C"]))
    g = synth.rng(4)
    Y = g.standard_normal((n, lam))
    order = g.permutation(lam)
    pv = O.params(n, lam, variant="separable")
    ps_ = O.params(n, lam)
    ps_.c1, ps_.cmu = pv.c1, pv.cmu
    full = O.covariance_update(Cd, st["p_c"], Y, order, ps_, 1.0)
    sep = O.covariance_update(Cd, st["p_c"], Y, order, pv, 1.0)
    assert np.count_nonzero(sep - np.diag(np.diag(sep))) == 0
    assert np.max(np.abs(np.diag(sep) - np.diag(full))) <= 1e-15 * np.max(np.diag(full))


def test_separable_stays_diagonal_and_converges_on_the_ellipsoid():
    n = 20
    st = O.new_descent(n, 0 or O.default_lambda(n), 2.0, 3, variant="separable")
    obj = O.Objective("ellipsoid", None, synth.optimum(n, 1))
    while not st.stop:
        O.generation(st, obj, so=O.StopOptions(max_gens=6000))
        assert np.count_nonzero(st.C - np.diag(np.diag(st.C))) == 0
    assert st.f_best < 1e-8, (st.gen, st.f_best, st.stop)


def test_active_converges_on_the_rotated_ellipsoid_with_fewer_evaluations():
    n = 10
    evals = {"standard": [], "active": []}
    for seed in range(1, 6):
        R, xs = synth.problem(n, seed)
        for var in evals:
            st = O.new_descent(n, O.default_lambda(n), 2.0, seed, variant=var)
            while not st.stop:
                O.generation(st, O.Objective("ellipsoid", R, xs), so=O.StopOptions(max_gens=5000))
            assert st.f_best < 1e-8, (var, seed, st.gen)
            evals[var].append(st.evals)
    assert np.median(evals["active"]) < np.median(evals["standard"]), evals
