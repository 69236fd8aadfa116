"""The float32 GEMM tiles of the mixed precisions (sampling product of eq. (1),
rotated-objective product, split-k rank-mu product of eq. (3)) and their
tuner.  Every tile at every site must meet the mixed-path parity bar against
the FP64 oracle on shapes with ragged row, column and k tails; the sampling
product must be bit-identical across tiles (each output sums its k terms in
the same order whatever the block tile); the tuner must leave the search
state untouched and round-trip its cache."""

import json

import numpy as np
import pytest

import synth
from helpers import TOL, one_generation, rank_agreement, rel

pytestmark = pytest.mark.gpu

NUM_CONFIGS = 7  # CMAES_NUM_GEMM_CONFIGS


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_11765_amd as P
    assert P.cmaes_gemm_config_count() == NUM_CONFIGS
    return P


def _square(P, cfg):
    bm, bn, _ = P.cmaes_gemm_config_info(cfg)
    return bm == bn


@pytest.mark.parametrize("cfg", range(NUM_CONFIGS))
@pytest.mark.parametrize("n,lam", [(37, 53), (130, 301), (257, 1030)])
def test_tile_parity(P, cfg, n, lam):
    print(f"case tile cfg={cfg} {P.cmaes_gemm_config_info(cfg)} n={n} lam={lam}", flush=True)
    st = synth.random_state(n, lam, seed=n * 5 + lam, cond=100.0)
    R, xs = synth.problem(n, seed=n + 9)
    Z = synth.normal_matrix(n, lam, seed=lam * 13 + n)

    def configure(es):
        es.set_gemm_config("sample", cfg)
        es.set_gemm_config("fitness", cfg)
        es.set_gemm_config("syrk", cfg if _square(P, cfg) else 0)

    g, o, info = one_generation(P, st, Z, "ellipsoid", R, xs, "mixed", configure=configure)
    errs = {"m": rel(g["m"], o.m), "C": rel(g["C"], o.C), "sigma": abs(g["sigma"] - o.sigma) / o.sigma,
            "p_sigma": rel(g["p_sigma"], o.ps), "p_c": rel(g["p_c"], o.pc)}
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < TOL["mixed"], (k, v)
    f_ref = info["f"]
    assert np.max(np.abs(g["f"] - f_ref)) <= 2e-5 * np.max(np.abs(f_ref))
    assert rank_agreement(f_ref, g["order"], info["order"], 1e-4) == 0
    assert np.array_equal(g["C"], g["C"].T)


def test_sampling_product_bit_identical_across_tiles(P):
    n, lam = 257, 1030
    st = synth.random_state(n, lam, seed=77, cond=1e3)
    X = []
    for cfg in range(NUM_CONFIGS):
        es = P.CMAES(n, lam, 1.0, seed=5, precision="mixed")
        try:
            es.set_gemm_config("sample", cfg)
            es.set_state(st)
            X.append(es.ask())
        finally:
            es.close()
    for cfg in range(1, NUM_CONFIGS):
        assert np.array_equal(X[cfg], X[0]), cfg


def test_syrk_site_takes_square_tiles_only(P):
    es = P.CMAES(16, 8, 1.0, seed=1, precision="mixed")
    try:
        for cfg in range(NUM_CONFIGS):
            if _square(P, cfg):
                es.set_gemm_config("syrk", cfg)
                assert es.gemm_config("syrk") == cfg
            else:
                with pytest.raises(P.CmaesError):
                    es.set_gemm_config("syrk", cfg)
        with pytest.raises(P.CmaesError):
            es.set_gemm_config("sample", NUM_CONFIGS)
    finally:
        es.close()


@pytest.mark.parametrize("precision", ["mixed", "mixed_bf16x3", "fp64"])
def test_autotune_keeps_state_and_caches(P, precision, tmp_path):
    n, lam = 130, 301
    R, xs = synth.problem(n, seed=4)
    cache = str(tmp_path / "tiles.json")
    es = P.CMAES(n, lam, 2.0, seed=11, precision=precision, objective="rastrigin", R=R, xstar=xs)
    try:
        es.generation()
        es.generation()
        before = es.state()
        chosen = es.autotune(reps=2, cache=cache)
        after = es.state()
        for k, v in before.items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, after[k], equal_nan=True), k
            else:
                assert v == after[k] or (v != v and after[k] != after[k]), k
        us = es.last_tune_us
        for site, cfg in chosen.items():
            assert es.gemm_config(site) == cfg
        if precision == "fp64":
            assert np.all(us == -1.0)
        else:
            assert us[2, chosen["syrk"]] > 0 and us[1, chosen["fitness"]] > 0
            if precision == "mixed":
                assert us[0, chosen["sample"]] == us[0][us[0] > 0].min()
            else:
                assert np.all(us[0] == -1.0)
        es.generation()
        assert np.all(np.isfinite(es.state()["C"]))
    finally:
        es.close()
    table = json.load(open(cache))
    assert len(table) == 1
    es2 = P.CMAES(n, lam, 2.0, seed=12, precision=precision, objective="rastrigin", R=R, xstar=xs)
    try:
        assert es2.autotune(reps=2, cache=cache) == chosen
        assert not hasattr(es2, "last_tune_us")
        for site, cfg in chosen.items():
            assert es2.gemm_config(site) == cfg
    finally:
        es2.close()


@pytest.mark.parametrize("precision,cfg", [("fp64", 0)] + [("mixed", c) for c in range(NUM_CONFIGS)])
def test_integer_inputs_give_exact_fitness(P, precision, cfg):
    """Integer-valued operands make the sampling product and the fused
    fitness exact in both precisions and with every tile: B a signed
    permutation, D and z small integers, m integer, sigma = 1/2, the
    unrotated sphere (every x_i is a multiple of 1/2, every f a multiple of
    1/4 far below 2^24), so each f must equal the plain float64 sum of
    squares bit for bit and the ranks must equal a stable argsort."""
    n, lam = 37, 53
    g = synth.rng(91)
    perm = g.permutation(n)
    B = np.zeros((n, n))
    B[perm, np.arange(n)] = g.choice([-1.0, 1.0], n)
    D = g.integers(1, 4, n).astype(np.float64)
    st = {"n": n, "lambda": lam, "m": g.integers(-3, 4, n).astype(np.float64), "sigma": 0.5,
          "C": (B * D ** 2) @ B.T, "B": B, "D": D, "p_sigma": np.zeros(n), "p_c": np.zeros(n), "gen": 3}
    Z = g.integers(-4, 5, (n, lam)).astype(np.float64)
    with P.CMAES(n, lam, 1.0, seed=1, precision=precision, objective="sphere", xstar=np.zeros(n)) as es:
        if precision == "mixed":
            es.set_gemm_config("sample", cfg)
            es.set_gemm_config("fitness", cfg)
        es.set_state(st)
        es.generation_with_z(Z)
        s = es.state()
    X = st["m"][:, None] + 0.5 * (B @ (D[:, None] * Z))
    f = np.sum(X * X, axis=0)
    assert np.array_equal(s["f"], f)
    assert np.array_equal(s["order"], np.argsort(f, kind="stable"))


@pytest.mark.parametrize("n,lam", [(2, 5), (37, 53), (64, 128), (257, 512), (300, 1100)])
def test_integer_inputs_give_exact_fitness_bf16x3(P, n, lam):
    """The same exactness check for the bf16 x 3 sampling product: operands
    of at most two significant bits are bf16 numbers (lo = 0), so the three
    products sum exactly in float32.  The shapes cover a single partial tile,
    exact tile edges, a ragged edge in both dimensions, a launch of 8 tiles
    (one run per XCD) and one of 18 (plain order)."""
    g = synth.rng(92 + n)
    perm = g.permutation(n)
    B = np.zeros((n, n))
    B[perm, np.arange(n)] = g.choice([-1.0, 1.0], n)
    D = g.integers(1, 4, n).astype(np.float64)
    st = {"n": n, "lambda": lam, "m": g.integers(-3, 4, n).astype(np.float64), "sigma": 0.5,
          "C": (B * D ** 2) @ B.T, "B": B, "D": D, "p_sigma": np.zeros(n), "p_c": np.zeros(n), "gen": 3}
    Z = g.integers(-4, 5, (n, lam)).astype(np.float64)
    with P.CMAES(n, lam, 1.0, seed=1, precision="mixed_bf16x3", objective="sphere", xstar=np.zeros(n)) as es:
        es.set_state(st)
        es.generation_with_z(Z)
        s = es.state()
    X = st["m"][:, None] + 0.5 * (B @ (D[:, None] * Z))
    f = np.sum(X * X, axis=0)
    assert np.array_equal(s["f"], f)
    assert np.array_equal(s["order"], np.argsort(f, kind="stable"))
