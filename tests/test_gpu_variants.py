"""The CMA-ES variants on the device (the paper's future work, Sec. 5) against
the oracle's: the active covariance update (negative weights for the worse
ranks) and the separable, large-scale variant (diagonal C, y = D z).

* one generation from an injected state and z, both precisions, several
  shapes (odd and even lambda, ragged tiles): f element by element, ranks,
  then m, sigma, C and the paths normwise, as for the standard variant;
* whole runs: every seed reaches f < 1e-8 and the median evaluation count is
  within 15% of the oracle's on the same seeds (the two sides' trajectories
  separate once an eigendecomposition meets a repeated eigenvalue, so only
  the distributions are compared; 8 seeds, hence the wider margin).
"""

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


def _state(n, lam, seed, variant):
    st = synth.random_state(n, lam, seed=seed, cond=100.0)
    if variant == "separable":  # diagonal C, B = I
        d = synth.rng(seed + 9).uniform(0.5, 5.0, n)
        st["C"], st["B"], st["D"] = np.diag(d), np.eye(n), np.sqrt(d)
    return st


def _one_generation(P, variant, precision, n, lam, kind, rotated):
    st = _state(n, lam, n * 5 + lam, variant)
    R, xs = synth.problem(n, seed=n + 21) if rotated else (None, synth.optimum(n, n + 21))
    Z = synth.normal_matrix(n, lam, seed=lam * 3 + n)
    with P.CMAES(n, lam, 1.0, seed=1, precision=precision, objective=kind, R=R, xstar=xs,
                 variant=variant) as es:
        es.set_state(st)
        es.generation_with_z(Z)
        g = es.state()
    o = O.new_descent(n, lam, 1.0, 1, variant=variant)
    o.m, o.sigma, o.C, o.B, o.D = st["m"].copy(), st["sigma"], st["C"].copy(), st["B"].copy(), st["D"].copy()
    o.ps, o.pc, o.gen = st["p_sigma"].copy(), st["p_c"].copy(), st["gen"]
    info = O.generation(o, O.Objective(kind, R, xs), Z=Z)
    return g, o, info, st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("variant", ["active", "separable"])
@pytest.mark.parametrize("n,lam,kind,rotated", [(10, 10, "ellipsoid", True), (10, 11, "sphere", False),
                                                (37, 53, "rastrigin", True), (130, 301, "ellipsoid", True),
                                                (257, 1030, "ellipsoid", False)])
def test_variant_one_generation_parity(P, variant, precision, n, lam, kind, rotated):
    print(f"case {variant} {precision} n={n} lam={lam} {kind}", flush=True)
    g, o, info, st = _one_generation(P, variant, precision, n, lam, kind, rotated)
    ferr = np.abs(g["f"] - info["f"]) / np.maximum(np.abs(info["f"]), 1e-300)
    assert np.max(ferr) <= FTOL[precision], float(np.max(ferr))
    assert rank_agreement(info["f"], g["order"], info["order"], RANK_TAU[precision]) == 0
    tol = TOL[precision]
    errs = {"m": rel(g["m"], o.m), "C": rel(g["C"], o.C), "sigma": abs(g["sigma"] - o.sigma) / o.sigma,
            "p_sigma": rel(g["p_sigma"], o.ps), "p_c": rel(g["p_c"], o.pc)}
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)
    if variant == "separable":
        assert np.count_nonzero(g["C"] - np.diag(np.diag(g["C"]))) == 0
        assert np.array_equal(g["B"], np.eye(n))
        assert rel(g["D"], o.D) < tol


@pytest.mark.parametrize("variant,kind,rotated,n", [("active", "ellipsoid", True, 10),
                                                     ("separable", "ellipsoid", False, 20)])
def test_variant_whole_runs(P, variant, kind, rotated, n):
    gpu, ora = [], []
    for seed in range(1, 9):
        R, xs = synth.problem(n, seed)
        R = R if rotated else None
        with P.CMAES(n, 0, 2.0, seed=seed, precision="fp64", objective=kind, R=R, xstar=xs, variant=variant,
                     max_gens=6000) as es:
            while True:
                es.generation()
                s = es.state(False)
                if s["stop"]:
                    break
        assert s["f_best"] < 1e-8, (seed, s["stop_names"])
        gpu.append(s["evals"])
        o = O.new_descent(n, O.default_lambda(n), 2.0, seed, variant=variant)
        while not o.stop:
            O.generation(o, O.Objective(kind, R, xs), so=O.StopOptions(max_gens=6000))
        assert o.f_best < 1e-8
        ora.append(o.evals)
    mg, mo = np.median(gpu), np.median(ora)
    print(f"{variant} median evals gpu {mg} oracle {mo}", flush=True)
    assert abs(mg - mo) <= 0.15 * mo


def test_variant_option_checks(P):
    with P.CMAES(8, 8, 1.0, seed=1) as es:
        opt = P.cmaes_get_options(es.h)
        opt.variant = 3
        with pytest.raises(P.CmaesError) as e:
            P.cmaes_set_options(es.h, opt)
        assert e.value.code == P.binding.CMAES_EINVAL
    with P.CMAES(8, 8, 1.0, seed=1, objective="sphere") as es:
        es.generation()
        opt = P.cmaes_get_options(es.h)
        opt.variant = 1
        with pytest.raises(P.CmaesError) as e:
            P.cmaes_set_options(es.h, opt)
        assert e.value.code == P.binding.CMAES_ESTATE
