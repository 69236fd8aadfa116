"""Shared helpers for the GPU parity tests: run one generation from an
injected state and injected z on both the HIP path (through the C ABI) and
the FP64 oracle, and measure normwise relative errors."""

from __future__ import annotations

import numpy as np

import oracle as O

TOL = {"fp64": 1e-12, "mixed": 1e-5}
# fitness values, element by element, relative to |f_i|
FTOL = {"fp64": 1e-12, "mixed": 5e-6}
# ranks must agree wherever neighbouring fitness gaps exceed tau * |f|
# (at least twice the fitness tolerance: below that two values may swap)
RANK_TAU = {"fp64": 1e-12, "mixed": 1e-5}


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def oracle_state(st: dict, sigma0=1.0, seed=1, kappa=0) -> O.State:
    o = O.new_descent(st["n"], st["lambda"], sigma0, seed, kappa=kappa)
    o.m, o.sigma, o.C = st["m"].copy(), float(st["sigma"]), st["C"].copy()
    o.B, o.D = st["B"].copy(), st["D"].copy()
    o.ps, o.pc, o.gen = st["p_sigma"].copy(), st["p_c"].copy(), int(st["gen"])
    return o


def one_generation(P, st, Z, kind, R, xs, precision, kappa=0, configure=None):
    """Returns (gpu_state, oracle_state, oracle_info); configure(es) runs on the
    device handle before the generation."""
    n, lam = st["n"], st["lambda"]
    es = P.CMAES(n, lam, 1.0, seed=1, precision=precision, objective=kind, R=R, xstar=xs,
                 eigen_interval=kappa)
    try:
        if configure is not None:
            configure(es)
        es.set_state(st)
        es.generation_with_z(Z)
        g = es.state()
    finally:
        es.close()
    o = oracle_state(st, kappa=kappa)
    info = O.generation(o, O.Objective(kind, R, xs), Z=Z)
    return g, o, info


def rank_agreement(f_ref, order_gpu, order_ref, tau):
    """Ranks must agree wherever neighbouring fitness gaps exceed tau*|f|."""
    fs = np.asarray(f_ref)[order_ref]
    bad = 0
    for r in range(len(fs)):
        lo = abs(fs[r] - fs[r - 1]) > tau * max(abs(fs[r]), abs(fs[r - 1])) if r > 0 else True
        hi = abs(fs[r + 1] - fs[r]) > tau * max(abs(fs[r]), abs(fs[r + 1])) if r + 1 < len(fs) else True
        if lo and hi and order_gpu[r] != order_ref[r]:
            bad += 1
    return bad
