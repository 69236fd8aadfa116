"""Pins for the oracle's generation, eigendecomposition and restart loop.

Each test ties the oracle to something other than its own code: the paper's
eq. (2) written out point by point, closed-form eigenpairs, statistical
properties of eq. (1), invariances of a rank-based method, the stationary
length of the sigma path under random selection, linear convergence on the
sphere and the lambda doubling of Alg. 2.
"""

import math

import numpy as np
import pytest

import oracle as O


def _random_spd(n, rng, cond=1e3):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.logspace(0, math.log10(cond), n)
    return (Q * ev) @ Q.T


def _random_state(n, lam, seed, cond=1e2):
    rng = np.random.default_rng(seed)
    st = O.new_descent(n, lam, 1.3, seed)
    st.C = _random_spd(n, rng, cond)
    st.B, st.D, _ = O.eigen_canonical(st.C)
    st.m = rng.uniform(-2, 2, n)
    st.ps = rng.standard_normal(n) * 0.5
    st.pc = rng.standard_normal(n) * 0.1
    st.gen = 3
    return st, rng


# --------------------------------------------------------------------- eq. (2)

@pytest.mark.parametrize("n,lam", [(3, 6), (7, 11), (20, 40)])
def test_covariance_update_equals_eq2(n, lam):
    """Eq. (2): C <- C + cmu sum_{i=1}^{lam} w_rk(i) (y_i y_i^T - C) + c1 (pc pc^T - C),
    summed over every point with its rank weight (zero beyond mu), checked
    against the oracle's eq. (3)-form update with h_sigma = 1."""
    st, rng = _random_state(n, lam, 5)
    p = st.p
    Y = rng.standard_normal((n, lam))
    f = rng.standard_normal(lam)
    order = O.rank_order(f)
    rank = np.empty(lam, dtype=int)
    rank[order] = np.arange(lam)
    w_rank = np.zeros(lam)
    w_rank[:p.mu] = p.w
    C2 = st.C.copy()
    acc = np.zeros((n, n))
    for i in range(lam):
        wi = w_rank[rank[i]]
        for r in range(n):
            for c in range(n):
                acc[r, c] += wi * (Y[r, i] * Y[c, i] - st.C[r, c])
    for r in range(n):
        for c in range(n):
            C2[r, c] = st.C[r, c] + p.cmu * acc[r, c] + p.c1 * (st.pc[r] * st.pc[c] - st.C[r, c])
    C3 = O.covariance_update(st.C, st.pc, Y, order, p, hsig=1.0)
    assert np.abs(C3 - C2).max() <= 1e-13 * np.abs(C2).max()


def test_covariance_update_fixed_point_and_spd():
    st, rng = _random_state(6, 12, 9)
    p = st.p
    Y = rng.standard_normal((6, 12))
    order = np.arange(12)
    p0 = O.Params(**{**p.__dict__, "c1": 0.0, "cmu": 0.0})
    np.testing.assert_allclose(O.covariance_update(st.C, st.pc, Y, order, p0, 1.0), st.C,
                               rtol=0, atol=1e-15 * np.abs(st.C).max())
    Cn = O.covariance_update(st.C, st.pc, Y, order, p, 0.0)
    assert np.array_equal(Cn, Cn.T)
    assert np.linalg.eigvalsh(Cn).min() > 0


# ------------------------------------------------------------------ eigen

def test_eigen_2x2_closed_form():
    a, b, c = 3.0, 1.25, -0.5 + 2.0
    C = np.array([[a, b], [b, c]])
    B, D, ok = O.eigen_canonical(C)
    mid, rad = (a + c) / 2.0, math.hypot((a - c) / 2.0, b)
    np.testing.assert_allclose(D ** 2, [mid - rad, mid + rad], rtol=1e-15)
    # eigenvector of the larger eigenvalue is proportional to (b, lam - a)
    v = np.array([b, mid + rad - a]) / math.hypot(b, mid + rad - a)
    assert abs(abs(B[:, 1] @ v) - 1.0) < 1e-15
    assert ok


@pytest.mark.parametrize("n", [1, 5, 64, 200])
def test_eigen_reconstruction_and_canonical_form(n):
    C = _random_spd(n, np.random.default_rng(n), cond=1e6)
    B, D, ok = O.eigen_canonical(C)
    assert ok
    assert np.linalg.norm(B @ np.diag(D ** 2) @ B.T - C) <= 1e-12 * np.linalg.norm(C)
    assert np.abs(B.T @ B - np.eye(n)).max() <= 1e-12
    assert np.all(np.diff(D) >= 0)
    idx = np.argmax(np.abs(B), axis=0)
    assert np.all(B[idx, np.arange(n)] > 0)


def test_eigen_flags_indefinite():
    C = np.diag([1.0, -1e-3, 2.0])
    _, D, ok = O.eigen_canonical(C)
    assert not ok and D.min() == 0.0


# -------------------------------------------------------------- eq. (1)

def test_sample_covariance_is_sigma2_C():
    """Eq. (1) draws x ~ N(m, sigma^2 C): the sample covariance of y -> C."""
    n = 4
    st, rng = _random_state(n, 8, 21, cond=20.0)
    Ys = []
    for g in range(60):
        Z = O.normals(99, 0, g, n, 4000)
        Y, X = O.sample(st, Z)
        Ys.append(Y)
        np.testing.assert_allclose(X, st.m[:, None] + st.sigma * Y, rtol=0, atol=1e-13)
    Y = np.concatenate(Ys, axis=1)
    S = Y @ Y.T / Y.shape[1]
    N = Y.shape[1]
    tol = 6.0 * np.sqrt((np.outer(np.diag(st.C), np.diag(st.C)) + st.C ** 2) / N)
    assert np.all(np.abs(S - st.C) < tol)
    assert np.abs(Y.mean(axis=1)).max() < 6.0 * np.sqrt(np.diag(st.C).max() / N)


# ---------------------------------------------------------- invariances

def _copy(st):
    import copy
    return copy.deepcopy(st)


def test_invariance_to_monotone_transform():
    st, _ = _random_state(8, 10, 4)
    a, b = _copy(st), _copy(st)
    obj = O.Objective("rastrigin")
    for _ in range(6):
        O.generation(a, obj)
        O.generation(b, lambda X: np.exp(obj(X) / 50.0) * 3.0 - 7.0)
    for k in ("m", "C", "ps", "pc", "B", "D"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert a.sigma == b.sigma


def test_rotation_covariance():
    """Sphere is rotation invariant: rotating m, C, paths and B by Q and
    keeping z gives the rotated trajectory (one generation, before eigen)."""
    n, lam = 9, 12
    st, rng = _random_state(n, lam, 17)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    r = _copy(st)
    r.m, r.C, r.B = Q @ st.m, Q @ st.C @ Q.T, Q @ st.B
    r.ps, r.pc = Q @ st.ps, Q @ st.pc
    r.p.kappa = st.p.kappa = 10 ** 6     # no eigen step inside this generation
    Z = O.normals(5, 0, 0, n, lam)
    O.generation(st, O.Objective("sphere"), Z=Z)
    O.generation(r, O.Objective("sphere"), Z=Z)
    assert np.linalg.norm(r.m - Q @ st.m) < 1e-12 * np.linalg.norm(st.m)
    assert np.linalg.norm(r.C - Q @ st.C @ Q.T) < 1e-12 * np.linalg.norm(st.C)
    assert np.linalg.norm(r.ps - Q @ st.ps) < 1e-12 * np.linalg.norm(st.ps)
    assert np.linalg.norm(r.pc - Q @ st.pc) < 1e-12 * np.linalg.norm(st.pc)
    assert abs(r.sigma - st.sigma) < 1e-13 * st.sigma


def test_csa_neutral_under_random_selection():
    """With rank-neutral (random) fitness, p_sigma is N(0, I) in its stationary
    state, so E||p_sigma|| = chi_n and ln sigma has no drift."""
    n, lam = 12, 10
    st = O.new_descent(n, lam, 1.0, 3)
    rng = np.random.default_rng(0)
    norms, logs = [], []
    for g in range(3000):
        O.generation(st, lambda X: rng.standard_normal(X.shape[1]))
        if g >= 200:
            norms.append(np.linalg.norm(st.ps))
            logs.append(math.log(st.sigma))
    assert abs(np.mean(norms) / st.p.chin - 1.0) < 0.03
    drift = (logs[-1] - logs[0]) / len(logs)
    assert abs(drift) < 3e-3


# ------------------------------------------------------- convergence, IPOP

def test_sphere_linear_convergence_config1():
    gens = []
    for seed in range(1, 16):
        st = O.new_descent(10, 10, 2.0, seed, kappa=1)
        so = O.StopOptions(max_gens=2000)
        logf = []
        while True:
            info = O.generation(st, O.Objective("sphere"), so=so)
            logf.append(math.log10(max(info["f"].min(), 1e-300)))
            if st.stop:
                break
        assert st.stop & O.STOP_FTARGET and st.f_best < 1e-8
        gens.append(st.gen)
        # log10 f decreases linearly: slope over the second half close to the whole-run slope
        x = np.arange(len(logf))
        slope = np.polyfit(x[len(x) // 3:], np.asarray(logf)[len(x) // 3:], 1)[0]
        assert -0.15 < slope < -0.03
    assert 80 <= np.median(gens) <= 300


def test_ipop_lambda_doubling_and_kmax():
    so = O.StopOptions(f_target=-1.0)           # unreachable target: all descents run
    best, x, log = O.ipop(3, 6, 2.0, 5, O.Objective("rastrigin"), k_max=8, so=so,
                          max_gens_per_descent=15)
    assert [d["lam"] for d in log] == [6, 12, 24, 48]
    assert [d["K"] for d in log] == [1, 2, 4, 8]
    assert [d["restart"] for d in log] == [0, 1, 2, 3]
    assert best == min(d["f_best"] for d in log)
    assert abs(O.rot_rastrigin(x[:, None])[0] - best) < 1e-9


def test_ipop_stops_at_target():
    best, _, log = O.ipop(4, 8, 2.0, 2, O.Objective("sphere"), k_max=64)
    assert len(log) == 1 and best < 1e-8


# ------------------------------------------------------------- stop tests

def test_stop_tolx_condition_and_noeffect():
    st = O.new_descent(5, 8, 2.0, 1)
    st.sigma = 1e-13
    st.f_best = 1.0
    st.hist = [1.0]
    bits = O.stop_bits(st, np.ones(8), O.StopOptions(), True)
    assert bits & O.STOP_TOLX
    st = O.new_descent(5, 8, 2.0, 1)
    st.D = np.array([1e-8, 1, 1, 1, 1.0])
    assert O.stop_bits(st, np.ones(8), O.StopOptions(), True) & O.STOP_CONDITIONCOV
    st = O.new_descent(5, 8, 2.0, 1)
    st.m = np.full(5, 1e20)
    b = O.stop_bits(st, np.ones(8), O.StopOptions(), True)
    assert b & O.STOP_NOEFFECTCOORD and b & O.STOP_NOEFFECTAXIS


def test_stop_tolhistfun_on_flat_function():
    st = O.new_descent(4, 8, 2.0, 3)
    while not st.stop:
        O.generation(st, lambda X: np.full(X.shape[1], 5.0))
    hl = 10 + math.ceil(30 * 4 / 8)
    assert st.stop & O.STOP_TOLHISTFUN and st.stop & O.STOP_TOLFUN
    assert st.gen == hl


def test_nan_fitness_ranks_last():
    f = np.array([3.0, np.nan, 1.0, np.inf, 1.0])
    assert list(O.rank_order(f)) == [2, 4, 0, 1, 3]


def test_mean_is_weighted_recombination_of_best_points():
    """Alg. 1's mean update: the new m is the weighted average of the mu best
    sampled points, sum_i w_i x_{i:lam} (weights sum to one)."""
    st, _ = _random_state(11, 16, 8)
    info = O.generation(st, O.Objective("ellipsoid"))
    X, order = info["X"], info["order"]
    want = X[:, order[:st.p.mu]] @ st.p.w
    assert np.linalg.norm(st.m - want) <= 1e-13 * np.linalg.norm(want)
    f = info["f"]
    assert np.all(np.diff(f[order]) >= 0)


def test_paths_stationary_with_frozen_covariance():
    """With c1 = cmu = 0 (C frozen, non-identity) and random selection,
    y_w ~ N(0, C / mu_eff), so p_c is stationary N(0, C) and p_sigma, built
    from C^{-1/2} y_w, stationary N(0, I): E[p_c^T C^-1 p_c] = E||p_sigma||^2 = n.
    (n = 30 keeps the h_sigma stall below 1e-3 of the generations.)"""
    n, lam = 30, 12
    rng = np.random.default_rng(1)
    st = O.new_descent(n, lam, 1.0, 77)
    st.p.c1 = 0.0
    st.p.cmu = 0.0
    st.C = _random_spd(n, rng, cond=30.0)
    st.B, st.D, _ = O.eigen_canonical(st.C)
    Ci = np.linalg.inv(st.C)
    qc, qs = [], []
    for g in range(15000):
        O.generation(st, lambda X: rng.standard_normal(X.shape[1]))
        if g >= 200:
            qc.append(st.pc @ Ci @ st.pc)
            qs.append(st.ps @ st.ps)
    assert abs(np.mean(qc) / n - 1.0) < 0.05
    assert abs(np.mean(qs) / n - 1.0) < 0.05


def test_hsig_stall_rate_matches_chi_distribution():
    """h_sigma normalises ||p_sigma|| by its random-walk scale so that, under
    random selection, ||p_sigma|| / sqrt(1-(1-c_sigma)^(2(g+1))) ~ chi_n at
    every g; the stall rate is then P(chi_n > (1.4 + 2/(n+1)) E chi_n)."""
    from scipy.stats import chi2
    n, lam, runs = 10, 10, 1500
    rng = np.random.default_rng(3)
    stalls = {0: 0, 4: 0}
    for s in range(runs):
        st = O.new_descent(n, lam, 1.0, 1000 + s)
        for g in range(5):
            info = O.generation(st, lambda X: rng.standard_normal(X.shape[1]))
            if g in stalls:
                stalls[g] += info["hsig"] == 0.0
    thr = (1.4 + 2.0 / (n + 1)) * st.p.chin
    p = chi2.sf(thr ** 2, n)
    for g, k in stalls.items():
        assert abs(k / runs - p) < 4.0 * math.sqrt(p * (1 - p) / runs) + 2.0 / runs, (g, k, p)
