"""Plain FP64 CPU oracle of one IPOP-CMA-ES generation and of the restart loop.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Written from the paper
"Massively parallel CMA-ES with increasing population" (arXiv 2409.11765):

* Alg. 1 (Sec. 2.1): one CMA-ES iteration = sample lambda points, evaluate
  them, update (m, C, sigma, p_sigma, p_c); return the best sampled point.
* Eq. (1) (Sec. 2.1): x_k = m + sigma * B * D * z_k, z_k ~ N(0, I), B the
  orthonormal eigenvectors of C, D the square roots of its eigenvalues.
* Eq. (2) (Sec. 2.1) and its rewrite eq. (3) (Sec. 3.1): the rank-one plus
  rank-mu covariance update with rank-based weights summing to one.
* Alg. 2 (Sec. 2.2): IPOP restarts with lambda = K * lambda_start, K doubling
  up to K_max; the answer is the best sampled point over all descents.
* Sec. 4.1 (setup): at the start of each descent m is drawn uniformly in the
  search box and sigma is a quarter of the box width.

The paper prints no parameter formula, no step-size rule and no stopping
thresholds (it defers to the default settings of the reference C code and to
the usual stopping conditions).  Readings taken here, all of them shared with
the GPU path:

* parameters, weights, cumulation and step-size rules: the published CMA-ES
  tutorial (Hansen, arXiv:1604.00772) with positive weights only;
* h_sigma stall of p_c included (reduces to eq. (3) when h_sigma = 1);
* stopping tests: those of the original IPOP-CMA-ES paper (Auger & Hansen,
  CEC 2005) with thresholds given in ``StopOptions``;
* random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = seed and
  counter = (row/4, candidate, generation, restart), Box-Muller to normals.

Pins (tests under ``tests/`` that tie this file to something other than itself):

* ``philox4x32_10``  - rocRAND's header-only Philox engine, compiled on the host.
* ``box_muller``     - moments and a Kolmogorov-Smirnov test against N(0,1).
* ``params``         - closed forms: default lambda values of the workloads,
  sum w = 1, mu_eff, chi_n against the exact Gamma-function expectation.
* ``covariance_update`` - the paper's eq. (2) written out over all lambda
  points with rank weights (the oracle uses the eq. (3) form).
* ``eigen_canonical``   - reconstruction, orthogonality, 2x2 closed form.
* ``generation``     - invariance to monotone transforms of f, rotation
  covariance, sample covariance of y, CSA drift under random selection,
  linear convergence on the sphere.
* ``ipop``           - lambda sequence lambda_start * 2^k and K_max stop.
* ``params`` / ``covariance_update`` variants - active: C stays positive
  definite against the worst negative-rank steps (the alpha_posdef bound),
  the update written out entry by entry with C^{-1/2} from eigh, zero
  negative weights give the standard update; separable: n = 1 equals the
  standard variant, C stays diagonal and equals the diagonal of the standard
  update with the separable rates; both converge on the ellipsoid.
* ``sphere``, ``rot_ellipsoid``, ``rot_rastrigin`` - zero at x* under any
  rotation, the ellipsoid's axis scales 10^(6 (i-1)/(n-1)) along R^T e_i,
  Rastrigin = sum u^2 at integer u and 20.25 n at u = 1/2, n = 1 edge case.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "default_lambda", "Params", "params",
    "philox4x32_10", "u32_to_unit", "box_muller", "normals", "init_mean",
    "Objective", "sphere", "rot_ellipsoid", "rot_rastrigin",
    "State", "new_descent", "sample", "rank_order", "covariance_update",
    "eigen_canonical", "generation", "StopOptions", "stop_bits", "ipop", "VARIANTS",
    "krep_leaf_seed", "k_replicated",
    "STOP_TOLHISTFUN", "STOP_TOLFUN", "STOP_TOLX", "STOP_NOEFFECTAXIS",
    "STOP_NOEFFECTCOORD", "STOP_CONDITIONCOV", "STOP_FTARGET", "STOP_MAXGEN",
    "STOP_MAXEVALS", "STOP_NUMERIC",
]

# ---------------------------------------------------------------------------
# Strategy parameters (reading: CMA-ES tutorial defaults, positive weights)
# ---------------------------------------------------------------------------


def default_lambda(n: int) -> int:
    """Default population size 4 + floor(3 ln n) (tutorial default; the
    workloads' lambda_start values 10/17/19/24 for n = 10/100/200/1000)."""
    return 4 + int(math.floor(3.0 * math.log(n)))


@dataclass
class Params:
    n: int
    lam: int
    mu: int
    w: np.ndarray          # w_1..w_mu, positive, non-increasing, sum 1
    mueff: float
    cs: float
    ds: float
    cc: float
    c1: float
    cmu: float
    chin: float
    kappa: int             # eigendecomposition interval in generations
    variant: str = "standard"
    # weights of all lambda ranks: w_1..w_mu as above, then 0 (standard,
    # separable) or the negative weights of the active update
    w_all: np.ndarray | None = None
    sumw: float = 1.0      # sum of w_all (< 1 with negative weights)


VARIANTS = ("standard", "active", "separable")


def params(n: int, lam: int, kappa: int = 0, variant: str = "standard") -> Params:
    """Default strategy parameters for dimension n and population lam.

    The weights are the rank weights w_rk(i) of eq. (2): better points get
    larger weights and the weights sum to one (Sec. 2.1).  Points ranked
    beyond mu get weight zero (reading: no negative weights).
    kappa = 0 selects the automatic interval max(1, ceil(1/(10 n (c1+cmu)))).

    variant (the paper's future work, Sec. 5; readings of the CMA-ES tutorial,
    Hansen arXiv:1604.00772, and of Ros & Hansen, PPSN 2008):
    * "active": ranks beyond mu get negative weights in the covariance update
      only, w'_i = ln((lam+1)/2) - ln i scaled so that they sum to
      -min(1 + c1/cmu, 1 + 2 mueff^-/(mueff + 2), (1 - c1 - cmu)/(n cmu)),
      mueff^- = (sum w'^-)^2 / sum (w'^-)^2; mean, paths and the other
      rates are those of the standard variant;
    * "separable": C is kept diagonal (the large-scale variant sep-CMA-ES),
      c1 and cmu multiplied by (n + 2)/3 (cmu at most 1 - c1), B = I and
      D = sqrt(diag C) after every generation (kappa = 1).
    """
    if n < 1 or lam < 2:
        raise ValueError("need n >= 1 and lambda >= 2")
    if variant not in VARIANTS:
        raise ValueError(f"variant must be one of {VARIANTS}")
    mu = lam // 2
    i = np.arange(1, mu + 1, dtype=np.float64)
    wp = math.log((lam + 1) / 2.0) - np.log(i)
    w = wp / wp.sum()
    mueff = 1.0 / float(np.sum(w * w))
    cs = (mueff + 2.0) / (n + mueff + 5.0)
    ds = 1.0 + 2.0 * max(0.0, math.sqrt((mueff - 1.0) / (n + 1.0)) - 1.0) + cs
    cc = (4.0 + mueff / n) / (n + 4.0 + 2.0 * mueff / n)
    c1 = 2.0 / ((n + 1.3) ** 2 + mueff)
    cmu = min(1.0 - c1, 2.0 * (mueff - 2.0 + 1.0 / mueff) / ((n + 2.0) ** 2 + mueff))
    chin = math.sqrt(n) * (1.0 - 1.0 / (4.0 * n) + 1.0 / (21.0 * n * n))
    w_all = np.concatenate([w, np.zeros(lam - mu)])
    sumw = 1.0
    if variant == "separable":
        c1 = min(1.0, c1 * (n + 2.0) / 3.0)
        cmu = min(1.0 - c1, cmu * (n + 2.0) / 3.0)
        kappa = 1
    if variant == "active":
        wn = math.log((lam + 1) / 2.0) - np.log(np.arange(mu + 1, lam + 1, dtype=np.float64))
        wn = np.minimum(wn, 0.0)          # an odd lam leaves w'_{mu+1} = 0
        if np.any(wn < 0.0) and cmu > 0.0:   # (cmu = 0, e.g. lam = 2: no rank-mu term at all)
            mueff_neg = float(wn.sum() ** 2 / np.sum(wn * wn))
            alpha = min(1.0 + c1 / cmu, 1.0 + 2.0 * mueff_neg / (mueff + 2.0),
                        (1.0 - c1 - cmu) / (n * cmu))
            w_all[mu:] = alpha * wn / np.sum(np.abs(wn))
            sumw = float(np.sum(w_all))
    if kappa <= 0:
        kappa = max(1, int(math.ceil(1.0 / (10.0 * n * (c1 + cmu)))))
    return Params(n, lam, mu, w, mueff, cs, ds, cc, c1, cmu, chin, kappa, variant, w_all, sumw)


# ---------------------------------------------------------------------------
# Random numbers: Philox4x32-10 and Box-Muller (the z_k ~ N(0, I) of eq. (1))
# ---------------------------------------------------------------------------

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).

    Counter words c0..c3 and key words k0, k1 are uint32 values (arrays
    broadcast).  Each round multiplies c0 and c2 by the two Philox constants,
    keeps the 64-bit products as (hi, lo) pairs and returns
    (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1), hi(c0*M0) ^ c3 ^ k1, lo(c0*M0)); the key
    is advanced by the two Weyl constants between rounds.
    Returns four uint32 arrays.
    """
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3))
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    a = np.asarray(k0, dtype=np.uint64) & _MASK
    b = np.asarray(k1, dtype=np.uint64) & _MASK
    for r in range(10):
        p0 = _M0 * x0
        p1 = _M1 * x2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        x0, x1, x2, x3 = (hi1 ^ x1 ^ a) & _MASK, lo1, (hi0 ^ x3 ^ b) & _MASK, lo0
        if r < 9:
            a = (a + _W0) & _MASK
            b = (b + _W1) & _MASK
    return (x0.astype(np.uint32), x1.astype(np.uint32),
            x2.astype(np.uint32), x3.astype(np.uint32))


def u32_to_unit(u) -> np.ndarray:
    """Map a uint32 to the open interval (0, 1): (u + 1/2) / 2^32."""
    return (np.asarray(u, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def box_muller(u1, u2):
    """Box-Muller: two independent N(0,1) values from two uniforms in (0,1)."""
    rho = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * math.pi * u2
    return rho * np.cos(t), rho * np.sin(t)


def _seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.uint32(seed & 0xFFFFFFFF), np.uint32(seed >> 32)


def normals(seed: int, restart: int, gen: int, n: int, lam: int) -> np.ndarray:
    """The n x lam matrix [z_1 .. z_lam] of eq. (1) for one generation.

    Element (i, k) comes from the Philox block with counter
    (i // 4, k, gen, restart) and key = seed: words (r0, r1) give rows
    4j, 4j+1 and words (r2, r3) rows 4j+2, 4j+3 through Box-Muller.
    """
    k0, k1 = _seed_key(seed)
    nb = (n + 3) // 4
    j = np.arange(nb, dtype=np.uint64)[:, None]
    k = np.arange(lam, dtype=np.uint64)[None, :]
    r0, r1, r2, r3 = philox4x32_10(j, k, np.uint64(gen & 0xFFFFFFFF),
                                   np.uint64(restart & 0xFFFFFFFF), k0, k1)
    za, zb = box_muller(u32_to_unit(r0), u32_to_unit(r1))
    zc, zd = box_muller(u32_to_unit(r2), u32_to_unit(r3))
    Z = np.empty((4 * nb, lam), dtype=np.float64)
    Z[0::4], Z[1::4], Z[2::4], Z[3::4] = za, zb, zc, zd
    return Z[:n]


INIT_GEN_WORD = 0xFFFFFFFF  # counter word 2 reserved for descent initialisation


def init_mean(seed: int, restart: int, n: int, lo: float, hi: float) -> np.ndarray:
    """Initial mean of a descent, uniform in the box [lo, hi]^n (Sec. 4.1).

    Coordinate i uses word i % 4 of the Philox block with counter
    (i // 4, 0, 0xFFFFFFFF, restart) and key = seed.
    """
    k0, k1 = _seed_key(seed)
    nb = (n + 3) // 4
    j = np.arange(nb, dtype=np.uint64)
    r = philox4x32_10(j, 0, INIT_GEN_WORD, restart & 0xFFFFFFFF, k0, k1)
    u = np.empty(4 * nb, dtype=np.float64)
    for q in range(4):
        u[q::4] = u32_to_unit(r[q])
    return lo + (hi - lo) * u[:n]


# ---------------------------------------------------------------------------
# Objectives (synthetic stand-ins for the benchmark suite of Sec. 4.1)
# ---------------------------------------------------------------------------


def sphere(X, xstar=None):
    """f(x) = sum_i (x_i - x*_i)^2 for every column of X."""
    U = X if xstar is None else X - np.asarray(xstar)[:, None]
    return np.sum(U * U, axis=0)


def _rotate(X, R, xstar):
    U = X if xstar is None else X - np.asarray(xstar)[:, None]
    return U if R is None else np.asarray(R) @ U


def rot_ellipsoid(X, R=None, xstar=None):
    """f(x) = sum_i 10^(6 (i-1)/(n-1)) u_i^2 with u = R (x - x*)."""
    U = _rotate(X, R, xstar)
    n = U.shape[0]
    e = np.arange(n, dtype=np.float64) * (6.0 / (n - 1)) if n > 1 else np.zeros(1)
    return np.sum((10.0 ** e)[:, None] * U * U, axis=0)


def rot_rastrigin(X, R=None, xstar=None):
    """f(x) = 10 n + sum_i (u_i^2 - 10 cos(2 pi u_i)) with u = R (x - x*)."""
    U = _rotate(X, R, xstar)
    n = U.shape[0]
    return 10.0 * n + np.sum(U * U - 10.0 * np.cos(2.0 * math.pi * U), axis=0)


@dataclass
class Objective:
    kind: str                      # "sphere" | "ellipsoid" | "rastrigin"
    R: np.ndarray | None = None    # n x n rotation (None = identity)
    xstar: np.ndarray | None = None

    def __call__(self, X):
        if self.kind == "sphere":
            return sphere(_rotate(X, self.R, self.xstar))
        if self.kind == "ellipsoid":
            return rot_ellipsoid(X, self.R, self.xstar)
        if self.kind == "rastrigin":
            return rot_rastrigin(X, self.R, self.xstar)
        raise ValueError(self.kind)


# ---------------------------------------------------------------------------
# Descent state and one generation (Alg. 1 loop body)
# ---------------------------------------------------------------------------

STOP_TOLHISTFUN = 1 << 0
STOP_TOLFUN = 1 << 1
STOP_TOLX = 1 << 2
STOP_NOEFFECTAXIS = 1 << 3
STOP_NOEFFECTCOORD = 1 << 4
STOP_CONDITIONCOV = 1 << 5
STOP_FTARGET = 1 << 6
STOP_MAXGEN = 1 << 7
STOP_MAXEVALS = 1 << 8
STOP_NUMERIC = 1 << 9


@dataclass
class StopOptions:
    """Stopping thresholds (reading of the 'usual stopping conditions' of
    Sec. 2.2, taken from the original IPOP-CMA-ES paper)."""
    tol_hist_fun: float = 1e-12
    tol_fun: float = 1e-12
    tol_x_factor: float = 1e-12      # TolX = tol_x_factor * sigma0
    max_condition: float = 1e14
    f_target: float = 1e-8
    max_gens: int = 0                # 0 = no limit
    max_evals: int = 0               # 0 = no budget (Alg. 2 'budget')


@dataclass
class State:
    """Everything Alg. 1 carries between iterations, plus bookkeeping."""
    p: Params
    m: np.ndarray
    sigma: float
    C: np.ndarray
    B: np.ndarray
    D: np.ndarray
    ps: np.ndarray
    pc: np.ndarray
    sigma0: float
    seed: int = 0
    restart: int = 0
    gen: int = 0
    evals: int = 0
    f_best: float = math.inf
    x_best: np.ndarray | None = None
    hist: list = field(default_factory=list)
    stop: int = 0


def new_descent(n, lam, sigma0, seed, restart=0, box=(-4.0, 4.0), kappa=0, variant="standard") -> State:
    """Initialisation line of Alg. 1 / Alg. 2: m uniform in the box (Sec. 4.1),
    sigma = sigma0, C = B = D = I, both evolution paths zero."""
    p = params(n, lam, kappa, variant)
    m = init_mean(seed, restart, n, box[0], box[1])
    I = np.eye(n)
    return State(p=p, m=m, sigma=float(sigma0), C=I.copy(), B=I.copy(), D=np.ones(n),
                 ps=np.zeros(n), pc=np.zeros(n), sigma0=float(sigma0), seed=seed,
                 restart=restart)


def sample(st: State, Z: np.ndarray):
    """Eq. (1): y_k = B D z_k and x_k = m + sigma y_k, all k at once."""
    Y = st.B @ (st.D[:, None] * Z)
    X = st.m[:, None] + st.sigma * Y
    return Y, X


def rank_order(f) -> np.ndarray:
    """Candidates sorted by fitness, ascending; NaN counts as +inf; equal
    values keep candidate order (stable).  order[r] = candidate of rank r."""
    fk = np.where(np.isnan(f), np.inf, np.asarray(f, dtype=np.float64))
    return np.argsort(fk, kind="stable")


def covariance_update(C, pc, Y, order, p: Params, hsig: float, B=None, D=None):
    """Rank-one plus rank-mu update in the eq. (3) form:
    C <- a C + c1 pc pc^T + cmu * sum_{i<=mu} w_i y_{i:lam} y_{i:lam}^T,
    a = 1 - c1 - cmu + (1 - hsig) c1 cc (2 - cc).  With hsig = 1 this is
    exactly eq. (3) (and eq. (2), since the weights sum to one).

    active: the sum runs over all lam ranks with the signed weights, a uses
    sum_i w_i instead of 1, and a negative weight is scaled by
    n / ||C^{-1/2} y_{i:lam}||^2 with C^{-1/2} = B D^{-1} B^T of the C that
    sampled y (B, D given).  separable: the diagonal of the standard update."""
    delta = (1.0 - hsig) * p.c1 * p.cc * (2.0 - p.cc)
    if p.variant == "active":
        a = 1.0 - p.c1 - p.cmu * p.sumw + delta
        Ys = Y[:, order]
        wo = p.w_all.copy()
        neg = wo < 0.0
        if np.any(neg):
            Ci = B @ ((B.T @ Ys[:, neg]) / D[:, None])
            wo[neg] = wo[neg] * p.n / np.sum(Ci * Ci, axis=0)
        Cn = a * C + p.c1 * np.outer(pc, pc) + p.cmu * ((Ys * wo[None, :]) @ Ys.T)
        return 0.5 * (Cn + Cn.T)
    a = 1.0 - p.c1 - p.cmu + delta
    Ys = Y[:, order[:p.mu]]
    if p.variant == "separable":
        dn = a * np.diag(C) + p.c1 * pc * pc + p.cmu * ((Ys * Ys) @ p.w)
        return np.diag(dn)
    Cn = a * C + p.c1 * np.outer(pc, pc) + p.cmu * ((Ys * p.w[None, :]) @ Ys.T)
    return 0.5 * (Cn + Cn.T)


def eigen_canonical(C):
    """C = B diag(D)^2 B^T with orthonormal B (Sec. 2.1), canonicalised:
    eigenvalues ascending; each eigenvector's largest-magnitude entry is
    positive.  Returns (B, D, ok) where ok is False if C is not positive
    definite (D is then clipped at zero for that axis)."""
    Cs = 0.5 * (C + C.T)
    ev, V = np.linalg.eigh(Cs)
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[idx, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    V = V * sgn[None, :]
    ok = bool(ev[0] > 0.0)
    return V, np.sqrt(np.maximum(ev, 0.0)), ok


def stop_bits(st: State, f_gen, so: StopOptions, eig_ok: bool) -> int:
    """Stopping tests after a generation (reading of Sec. 2.2)."""
    p, n = st.p, st.p.n
    bits = 0
    hl = 10 + int(math.ceil(30.0 * n / p.lam))
    if len(st.hist) >= hl:
        h = np.asarray(st.hist[-hl:])
        if h.max() - h.min() < so.tol_hist_fun:
            bits |= STOP_TOLHISTFUN
        fin = np.where(np.isnan(f_gen), np.inf, f_gen)
        if max(h.max(), fin.max()) - min(h.min(), fin.min()) < so.tol_fun:
            bits |= STOP_TOLFUN
    tolx = so.tol_x_factor * st.sigma0
    if (st.sigma * np.sqrt(np.diag(st.C)).max() < tolx
            and st.sigma * np.abs(st.pc).max() < tolx):
        bits |= STOP_TOLX
    ax = st.gen % n
    if np.all(st.m == st.m + 0.1 * st.sigma * st.D[ax] * st.B[:, ax]):
        bits |= STOP_NOEFFECTAXIS
    if np.any(st.m == st.m + 0.2 * st.sigma * np.sqrt(np.diag(st.C))):
        bits |= STOP_NOEFFECTCOORD
    dmin, dmax = st.D.min(), st.D.max()
    if (not eig_ok) or dmin <= 0.0 or (dmax / dmin) ** 2 > so.max_condition:
        bits |= STOP_CONDITIONCOV
    if st.f_best < so.f_target:
        bits |= STOP_FTARGET
    if so.max_gens > 0 and st.gen >= so.max_gens:
        bits |= STOP_MAXGEN
    if so.max_evals > 0 and st.evals >= so.max_evals:
        bits |= STOP_MAXEVALS
    if not (np.all(np.isfinite(st.m)) and math.isfinite(st.sigma) and np.all(np.isfinite(st.C))):
        bits |= STOP_NUMERIC
    return bits


def generation(st: State, objective, Z=None, so: StopOptions | None = None, fvals=None):
    """One iteration of Alg. 1 on state st (modified in place).

    Z: the n x lam normal matrix (drawn from the Philox stream if None).
    fvals: optional precomputed fitness values (the ask/tell path).
    Returns a dict with the generation's Y, X, f and rank order.
    """
    p, n = st.p, st.p.n
    so = so or StopOptions()
    if Z is None:
        Z = normals(st.seed, st.restart, st.gen, n, p.lam)
    Y, X = sample(st, Z)                                           # eq. (1)
    f = np.asarray(objective(X) if fvals is None else fvals, dtype=np.float64)
    order = rank_order(f)                                          # rk(i)
    sel = order[:p.mu]
    yw = Y[:, sel] @ p.w                                           # weighted shift
    m_old, sigma_old = st.m, st.sigma
    st.m = m_old + sigma_old * yw                                  # mean update
    # C^{-1/2} y_w = B D^{-1} B^T y_w  (cumulation path for sigma)
    cinv_yw = st.B @ ((st.B.T @ yw) / st.D)
    st.ps = (1.0 - p.cs) * st.ps + math.sqrt(p.cs * (2.0 - p.cs) * p.mueff) * cinv_yw
    nps = float(np.linalg.norm(st.ps))
    hsig = 1.0 if nps / math.sqrt(1.0 - (1.0 - p.cs) ** (2 * (st.gen + 1))) \
        < (1.4 + 2.0 / (n + 1.0)) * p.chin else 0.0
    st.pc = (1.0 - p.cc) * st.pc + hsig * math.sqrt(p.cc * (2.0 - p.cc) * p.mueff) * yw
    st.C = covariance_update(st.C, st.pc, Y, order, p, hsig, st.B, st.D)  # eq. (2)/(3)
    st.sigma = sigma_old * math.exp((p.cs / p.ds) * (nps / p.chin - 1.0))
    st.gen += 1
    st.evals += p.lam
    eig_ok = True
    if p.variant == "separable":
        dc = np.diag(st.C)
        st.B, st.D, eig_ok = np.eye(n), np.sqrt(np.maximum(dc, 0.0)), bool(np.all(dc > 0.0))
    elif st.gen % p.kappa == 0:
        st.B, st.D, eig_ok = eigen_canonical(st.C)
    fin = np.where(np.isnan(f), np.inf, f)
    i0 = int(order[0])
    st.hist.append(float(fin[i0]))
    if fin[i0] < st.f_best:
        st.f_best = float(fin[i0])
        st.x_best = X[:, i0].copy()
    st.stop = stop_bits(st, f, so, eig_ok)
    return {"Y": Y, "X": X, "f": f, "order": order, "yw": yw, "hsig": hsig, "Z": Z}


# ---------------------------------------------------------------------------
# IPOP restart loop (Alg. 2)
# ---------------------------------------------------------------------------


def ipop(n, lam_start, sigma0, seed, objective, k_max=2 ** 9, box=(-4.0, 4.0),
         so: StopOptions | None = None, kappa=0, max_total_evals=0, max_gens_per_descent=0,
         variant="standard"):
    """Alg. 2: K = 1; while K <= K_max and budget left: fresh descent with
    lambda = K * lambda_start until a stopping test fires; K <- 2K.
    Returns (best f, best x, list of per-descent records)."""
    so = so or StopOptions()
    K, restart = 1, 0
    best_f, best_x, evals, log = math.inf, None, 0, []
    while K <= k_max and (max_total_evals <= 0 or evals < max_total_evals):
        st = new_descent(n, K * lam_start, sigma0, seed, restart, box, kappa, variant)
        so_d = StopOptions(**{**so.__dict__, "max_gens": max_gens_per_descent or so.max_gens})
        while True:
            generation(st, objective, so=so_d)
            if st.stop:
                break
        evals += st.evals
        if st.f_best < best_f:
            best_f, best_x = st.f_best, st.x_best
        log.append({"K": K, "lam": st.p.lam, "restart": restart, "gens": st.gen,
                    "evals": st.evals, "f_best": st.f_best, "stop": st.stop})
        if best_f < so.f_target:
            break
        K *= 2
        restart += 1
    return best_f, best_x, log


# ---------------------------------------------------------------------------
# K-Replicated strategy (Alg. 3, Sec. 3.2.2) on one machine
# ---------------------------------------------------------------------------

_U64 = (1 << 64) - 1


def krep_leaf_seed(seed: int, j: int) -> int:
    """Seed of leaf j of the tree (reading: the run's seed mixed with the leaf
    index by two odd 64-bit multipliers, so that leaves draw distinct
    streams)."""
    return (int(seed) * 0x9E3779B97F4A7C15 + j * 0xBF58476D1CE4E5B9 + 1) & _U64


def k_replicated(n, lam_start, k_max, sigma0, seed, objective, so: StopOptions | None = None,
                 box=(-4.0, 4.0), kappa=0, max_lockstep=100000):
    """Alg. 3 with the processes replaced by lockstep generations: k_max leaf
    descents with lam_start each start together; a generation steps every
    running descent once; when both children of a tree node have stopped,
    the node's descent starts with twice their population (it continues the
    left child's stream at the next restart index, with the left child's
    lambda doubled) and the children are done; the run ends when the root
    stops or the best f of any descent falls below f_target.

    Returns (best f, total evaluations, lockstep generations, per-node log)."""
    so = so or StopOptions()
    levels = int(round(math.log2(k_max)))
    assert 1 << levels == k_max, "k_max must be a power of two"
    # node (level l, index j) holds [state, finished, lam, seed, restart]
    nodes = {}
    for j in range(k_max):
        s = krep_leaf_seed(seed, j)
        nodes[(0, j)] = [new_descent(n, lam_start, sigma0, s, 0, box, kappa), False, lam_start, s, 0]
    best, evals, gens, log = math.inf, 0, 0, []
    while gens < max_lockstep:
        running = [k for k, v in sorted(nodes.items()) if not v[1]]
        for k in running:
            st = nodes[k][0]
            generation(st, objective, so=so)
            evals += st.p.lam
            best = min(best, st.f_best)
            if st.stop:
                nodes[k][1] = True
                log.append({"node": k, "lam": st.p.lam, "gens": st.gen, "f_best": st.f_best, "stop": st.stop})
        gens += 1
        for l in range(1, levels + 1):
            for j in range(k_max >> l):
                a, b = (l - 1, 2 * j), (l - 1, 2 * j + 1)
                if (l, j) in nodes or not (nodes.get(a, [None, False])[1] and nodes.get(b, [None, False])[1]):
                    continue
                _, _, lam_a, s_a, r_a = nodes[a]
                nodes[(l, j)] = [new_descent(n, 2 * lam_a, sigma0, s_a, r_a + 1, box, kappa), False,
                                 2 * lam_a, s_a, r_a + 1]
        root = nodes.get((levels, 0))
        if (root is not None and root[1]) or best < so.f_target:
            break
    return best, evals, gens, log
