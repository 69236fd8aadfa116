"""Ranking (Alg. 1: the candidates sorted by fitness, rk(i) in Sec. 2.1)
through the C ABI's ask/tell path: the device permutation must equal, index
for index, the stable ascending order of the told values with NaN ranked as
+inf and -0 tied with +0.  The sizes cover a single sorted chunk of 256
keys (no merge), ragged last chunks, one and several merge groups of 8
chunks, and lambda = 20011 (79 chunks, 10 groups)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_11765_amd as P
    return P


def _expected(f):
    key = np.where(np.isnan(f), np.inf, f) + 0.0  # -0 + 0 = +0
    return np.argsort(key, kind="stable")


def _values(lam, rng, kind):
    if kind == "distinct":
        return rng.standard_normal(lam)
    if kind == "ties":
        return rng.integers(0, 7, lam).astype(np.float64)
    # special values mixed into a tied background
    f = rng.integers(-3, 4, lam).astype(np.float64)
    specials = np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, np.nan, 1e308, -1e308, 5e-324])
    pos = rng.choice(lam, size=min(lam, 3 * len(specials)), replace=False)
    f[pos] = np.resize(specials, len(pos))
    return f


@pytest.mark.parametrize("lam", [2, 3, 5, 100, 1000, 6144, 8191, 8192, 8193, 9728, 20011])
@pytest.mark.parametrize("kind", ["distinct", "ties", "special"])
def test_device_rank_is_the_stable_order(P, lam, kind):
    print(f"case rank lam={lam} {kind}", flush=True)
    n = 4
    rng = np.random.default_rng(lam * 31 + len(kind))
    f = _values(lam, rng, kind)
    with P.CMAES(n, lam, 1.0, seed=3, precision="fp64") as es:
        es.ask()
        es.tell(f)
        order = es.state()["order"]
    assert np.array_equal(order, _expected(f))
