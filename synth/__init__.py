"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds no CMA-ES arithmetic: only reproducible random problem instances (the
synthetic stand-ins for the benchmark suite of the paper's Sec. 4.1) and
random descent states / normal matrices that tests inject into both the HIP
path and the oracle.  Every generator is numpy PCG64 seeded explicitly.
"""

from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar_rotation(n: int, seed: int) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix: QR of a standard Gaussian
    matrix with the columns' signs fixed by the diagonal of the triangular
    factor (Mezzadri's recipe)."""
    G = rng(seed).standard_normal((n, n))
    Q, Rq = np.linalg.qr(G)
    return Q * np.sign(np.diag(Rq))[None, :]


def optimum(n: int, seed: int, lo: float = -4.0, hi: float = 4.0) -> np.ndarray:
    """x* uniform in the search box, from a stream distinct from R's."""
    return rng(seed + 0x5EED).uniform(lo, hi, n)


def problem(n: int, seed: int):
    """(R, x*) of a rotated synthetic objective instance."""
    return haar_rotation(n, seed), optimum(n, seed)


def normal_matrix(n: int, lam: int, seed: int) -> np.ndarray:
    """An n x lambda matrix of independent N(0, 1) values to inject as z."""
    return rng(seed).standard_normal((n, lam))


def random_state(n: int, lam: int, seed: int, cond: float = 100.0, sigma: float = 0.7, gen: int = 3):
    """A non-trivial descent state built from its eigenpairs: C = B diag(D^2) B^T
    with a Haar B whose columns are sign-normalised (largest entry positive),
    eigenvalues log-spaced in [1, cond] (ascending), random m and paths."""
    g = rng(seed)
    B = haar_rotation(n, seed + 1)
    idx = np.argmax(np.abs(B), axis=0)
    B = B * np.sign(B[idx, np.arange(n)])[None, :]
    ev = np.logspace(0.0, np.log10(cond), n) if n > 1 else np.ones(1)
    D = np.sqrt(ev)
    C = (B * ev[None, :]) @ B.T
    C = 0.5 * (C + C.T)
    return {"n": n, "lambda": lam, "m": g.uniform(-2.0, 2.0, n), "sigma": sigma, "C": C, "B": B, "D": D,
            "p_sigma": 0.5 * g.standard_normal(n), "p_c": 0.1 * g.standard_normal(n), "gen": gen}
