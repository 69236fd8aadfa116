"""GPU tests of the batched concurrent descents (K-Distributed, Sec. 3.2.3):
a batch instance evolves bit-identically to the same descent run alone, every
instance of the concurrent-restart workload (n = 200, lambda_k = 19 * 2^k)
matches the oracle's first generation from the same seed, stopped instances
restart with the same population size, and the workload runs."""

import numpy as np
import pytest

import oracle as O
import synth
from helpers import FTOL, RANK_TAU, TOL, rank_agreement, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_11765_amd as P
    return P


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_bf16x3"])
def test_batch_instance_equals_solo_run(P, precision):
    ns, lams, seeds = [10, 37, 64], [10, 20, 40], [5, 6, 7]
    sig = [2.0, 1.5, 1.0]
    gens = 6
    with P.CMAESBatch(ns, lams, sig, seeds, precision=precision, eigen_interval=1) as b:
        for k, n in enumerate(ns):
            R, xs = synth.problem(n, 100 + k)
            b.set_objective(k, "rastrigin", R, xs)
        for _ in range(gens):
            b.generation()
        got = [b.state(k) for k in range(len(ns))]
    for k, n in enumerate(ns):
        R, xs = synth.problem(n, 100 + k)
        with P.CMAES(n, lams[k], sig[k], seed=seeds[k], precision=precision, objective="rastrigin", R=R,
                     xstar=xs, eigen_interval=1) as es:
            # the batch's grouped eigensolve closes with sweeps only
            es.set_eigen_correction(False)
            for _ in range(gens):
                es.generation()
            want = es.state()
        for key in ("m", "C", "B", "D", "p_sigma", "p_c", "f"):
            assert np.array_equal(got[k][key], want[key]), (k, key)
        assert got[k]["sigma"] == want["sigma"] and got[k]["gen"] == want["gen"] == gens


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_of_uneven_block_sizes_equals_solo_runs(P, precision):
    """Descents whose padded sizes differ (N = 64, 128 and 160: 3, 7 and 9
    rounds per sweep) share one grouped eigensolve, each deciding its sweeps
    at its own rounds; every one must still evolve exactly as it does alone
    (n > 64 alone takes the single-descent block path)."""
    ns, lams, seeds = [40, 100, 130], [12, 20, 24], [21, 22, 23]
    sig = [2.0, 1.5, 1.0]
    gens = 5
    with P.CMAESBatch(ns, lams, sig, seeds, precision=precision, eigen_interval=1) as b:
        for k, n in enumerate(ns):
            R, xs = synth.problem(n, 200 + k)
            b.set_objective(k, "rastrigin", R, xs)
        for _ in range(gens):
            b.generation()
        got = [b.state(k) for k in range(len(ns))]
    for k, n in enumerate(ns):
        R, xs = synth.problem(n, 200 + k)
        with P.CMAES(n, lams[k], sig[k], seed=seeds[k], precision=precision, objective="rastrigin", R=R,
                     xstar=xs, eigen_interval=1) as es:
            es.set_eigen_correction(False)
            for _ in range(gens):
                es.generation()
            want = es.state()
        for key in ("m", "C", "B", "D", "p_sigma", "p_c", "f"):
            assert np.array_equal(got[k][key], want[key]), (k, key)
        assert got[k]["sigma"] == want["sigma"] and got[k]["gen"] == want["gen"] == gens


def test_batch_restart_on_finish_keeps_lambda(P):
    with P.CMAESBatch([12, 12], [8, 16], [2.0, 2.0], [1, 2], precision="fp64", max_gens=3) as b:
        for k in range(2):
            b.set_objective(k, "sphere")
        for _ in range(4):
            b.generation()
        s = [b.state(k, arrays=False) for k in range(2)]
        f, kb = b.best()
    for k, lam in enumerate([8, 16]):
        assert s[k]["lambda"] == lam
        assert s[k]["restart"] == 1          # stopped after 3 generations, restarted once
        assert s[k]["gen"] == 1              # one generation into the new descent
        assert s[k]["total_evals"] == 4 * lam
    assert kb in (0, 1) and f == min(s[0]["f_best"], s[1]["f_best"])


def test_grouped_batch_restart_on_finish_and_best(P):
    """The same on the grouped front (mixed precision, rotated objectives):
    the stop bits and f_best the host reads after a batch generation come
    from the stop kernel's mapped copy, and must agree with each descent's
    state."""
    ns, lams = [12, 30], [8, 16]
    with P.CMAESBatch(ns, lams, [2.0, 2.0], [1, 2], precision="mixed", max_gens=3) as b:
        for k, n in enumerate(ns):
            R, xs = synth.problem(n, 40 + k)
            b.set_objective(k, "rastrigin", R, xs)
        f0, k0 = b.best()
        assert k0 == -1 and f0 == np.inf    # no generation yet
        for g in range(4):
            b.generation()
            s = [b.state(k, arrays=False) for k in range(2)]
            f, kb = b.best()
            assert f == min(s[0]["f_best"], s[1]["f_best"]) and s[kb]["f_best"] == f
    for k, lam in enumerate(lams):
        assert s[k]["lambda"] == lam
        assert s[k]["restart"] == 1
        assert s[k]["gen"] == 1
        assert s[k]["total_evals"] == 4 * lam


def test_concurrent_restart_workload_runs(P):
    """10 instances, n = 200, lambda_k = 19 * 2^k (k = 0..9), rotated Rastrigin
    with per-instance seeds, mixed precision."""
    K, n = 10, 200
    lams = [19 * 2 ** k for k in range(K)]
    seeds = [100 + k for k in range(K)]
    with P.CMAESBatch([n] * K, lams, [2.0] * K, seeds, precision="mixed") as b:
        for k in range(K):
            R, xs = synth.problem(n, seeds[k])
            b.set_objective(k, "rastrigin", R, xs)
        for _ in range(3):
            b.generation()
        for k in range(K):
            s = b.state(k)
            assert s["lambda"] == lams[k] and s["total_evals"] == 3 * lams[k]
            assert np.all(np.isfinite(s["m"])) and np.isfinite(s["sigma"])
            C, B, D = s["C"], s["B"], s["D"]
            assert np.max(np.abs(B.T @ B - np.eye(n))) <= 1e-12
            if s["gen"] % s["kappa"] == 0:   # the decomposition ran in this generation
                assert np.linalg.norm(B @ np.diag(D ** 2) @ B.T - C) <= 1e-12 * np.linalg.norm(C)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_concurrent_restart_workload_first_generation_matches_oracle(P, precision):
    """One batch generation of the 10 uneven instances (n = 200, lambda_k =
    19 * 2^k, seeds 100 + k, rotated Rastrigin) against the oracle's first
    generation of each descent: both start from the seed's mean with C = I and
    draw the same Philox z (float32-rounded in the mixed path), so f element by
    element, the ranks (wherever fitness gaps exceed the rank tolerance), m,
    sigma, C and both paths must agree to the path's tolerance."""
    K, n = 10, 200
    lams = [19 * 2 ** k for k in range(K)]
    seeds = [100 + k for k in range(K)]
    with P.CMAESBatch([n] * K, lams, [2.0] * K, seeds, precision=precision) as b:
        for k in range(K):
            R, xs = synth.problem(n, seeds[k])
            b.set_objective(k, "rastrigin", R, xs)
        b.generation()
        got = [b.state(k) for k in range(K)]
    for k in range(K):
        print(f"case batch instance k={k} lambda={lams[k]} {precision}", flush=True)
        R, xs = synth.problem(n, seeds[k])
        o = O.new_descent(n, lams[k], 2.0, seeds[k])
        Z = O.normals(seeds[k], 0, 0, n, lams[k])
        if precision == "mixed":
            Z = Z.astype(np.float32).astype(np.float64)
        info = O.generation(o, O.Objective("rastrigin", R, xs), Z=Z)
        g = got[k]
        assert g["gen"] == 1 and g["lambda"] == lams[k]
        ferr = np.abs(g["f"] - info["f"]) / np.abs(info["f"])
        assert np.max(ferr) <= FTOL[precision], (k, float(np.max(ferr)))
        assert rank_agreement(info["f"], g["order"], info["order"], RANK_TAU[precision]) == 0, k
        if precision != "fp64":
            # float32 fitness can reorder near-ties (allowed by the check
            # above); the update arithmetic is compared for the device's
            # ranking by driving the oracle with the device's fitness values
            o = O.new_descent(n, lams[k], 2.0, seeds[k])
            O.generation(o, None, Z=Z, fvals=g["f"])
        errs = {"m": rel(g["m"], o.m), "C": rel(g["C"], o.C), "sigma": abs(g["sigma"] - o.sigma) / o.sigma,
                "p_sigma": rel(g["p_sigma"], o.ps), "p_c": rel(g["p_c"], o.pc)}
        for key, v in errs.items():
            assert v < TOL[precision], (k, key, v)
