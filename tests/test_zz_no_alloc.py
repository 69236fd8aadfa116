"""cmaes_ask_noalloc, the allocation-free variant of cmaes_ask: called through
the C ABI, its points must equal cmaes_ask's bit for bit (same seed, state
and generation), on two calls in a row with the second smaller, and it must
not allocate (every allocation of a handle built with the allocator hook is
counted); sizes beyond its static staging area are refused."""

import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_11765_amd as P
    return P


def _ask(P, name, es, n, lam):
    X = np.full((n, lam), np.nan, order="F")
    rc = getattr(P.library(), name)(es.h, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, P.cmaes_last_error()
    return X


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ask_noalloc_equals_ask(P, precision):
    for n, lam in ((40, 96), (17, 24)):            # the second call is smaller
        print(f"case ask_noalloc {precision} n={n} lam={lam}", flush=True)
        st = synth.random_state(n, lam, seed=n + lam, gen=2)
        out = {}
        for name in ("cmaes_ask", "cmaes_ask_noalloc"):
            with P.CMAES(n, lam, 1.5, seed=7, precision=precision, allocator="torch") as es:
                es.set_state(st)
                before = len(es.allocator.live)
                X = _ask(P, name, es, n, lam)
                grew = len(es.allocator.live) - before
                # the points and the rest of the generation
                f = np.sum(X * X, axis=0)
                es.tell(f)
                out[name] = (X, es.state(), grew)
        Xa, sa, grew_a = out["cmaes_ask"]
        Xb, sb, grew_b = out["cmaes_ask_noalloc"]
        assert grew_a == 1 and grew_b == 0          # cmaes_ask allocates its staging buffer once
        assert np.all(np.isfinite(Xb))
        assert np.array_equal(Xa, Xb)
        for k in ("m", "C", "p_sigma", "p_c"):
            assert np.array_equal(sa[k], sb[k]), k


def test_ask_noalloc_repeated_calls_share_the_staging_area(P):
    n, lam = 30, 50
    with P.CMAES(n, lam, 1.0, seed=3, precision="mixed") as a, P.CMAES(n, lam, 1.0, seed=3, precision="mixed") as b:
        a.state(arrays=False)
        b.state(arrays=False)
        for _ in range(3):
            Xa = _ask(P, "cmaes_ask", a, n, lam)
            Xb = _ask(P, "cmaes_ask_noalloc", b, n, lam)
            assert np.array_equal(Xa, Xb)
            f = np.sum((Xa - 1.0) ** 2, axis=0)
            a.tell(f)
            b.tell(f)


def test_ask_noalloc_refusals(P):
    lib = P.library()
    X = np.zeros((4, 4), order="F")
    xp = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    # buffers not created yet: refused, nothing allocated
    with P.CMAES(4, 4, 1.0, seed=1) as es:
        assert lib.cmaes_ask_noalloc(es.h, xp) == P.binding.CMAES_ESTATE
        assert lib.cmaes_ask_noalloc(es.h, None) == P.binding.CMAES_EINVAL
    # beyond the staging area (n * lambda > 2^20 doubles)
    with P.CMAES(1100, 1000, 1.0, seed=1) as es:
        es.state(arrays=False)
        assert lib.cmaes_ask_noalloc(es.h, xp) == P.binding.CMAES_EINVAL
        assert "exceeds" in P.cmaes_last_error()
