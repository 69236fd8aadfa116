"""The C ABI's contract, on the device (through ctypes, as any C caller):

* caller buffers are consumed before a call returns: the z matrix of
  cmaes_generation_with_z and the fitness values of cmaes_tell are
  overwritten with NaN right after the call, and the result must still match
  the oracle;
* a stopped descent refuses cmaes_generation / cmaes_ask with CMAES_ESTATE
  until a restart or cmaes_set_state clears the stop;
* a generation whose eigendecomposition meets non-finite values returns
  CMAES_ENUMERIC with the stop bits set;
* the allocator hook: every device buffer from PyTorch's caching allocator,
  results bit-identical to hipMalloc's, and the hook fixed after the first
  allocation.
"""

import ctypes

import numpy as np
import pytest

import oracle as O
import synth
from helpers import TOL, oracle_state, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_11765_amd as P
    return P


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_injected_z_is_consumed_before_the_call_returns(P, precision):
    n, lam = 200, 19            # kappa = 3: no eigen step at generation 3 -> 4
    print(f"case z hand-off {precision}", flush=True)
    st = synth.random_state(n, lam, seed=n * 7 + lam, cond=100.0)
    R, xs = synth.problem(n, seed=n + 3)
    Z = synth.normal_matrix(n, lam, seed=lam * 11 + n)
    lib = P.library()
    with P.CMAES(n, lam, 1.0, seed=1, precision=precision, objective="ellipsoid", R=R, xstar=xs) as es:
        es.set_state(st)
        Zf = np.array(Z, dtype=np.float64, order="F")
        rc = lib.cmaes_generation_with_z(es.h, Zf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        Zf[:] = np.nan          # the library must not read the buffer any more
        assert rc == 0, P.cmaes_last_error()
        g = es.state()
    o = oracle_state(st)
    O.generation(o, O.Objective("ellipsoid", R, xs), Z=Z)
    assert np.all(np.isfinite(g["f"]))
    for k, a, b in (("m", g["m"], o.m), ("C", g["C"], o.C), ("p_c", g["p_c"], o.pc)):
        assert rel(a, b) < TOL[precision], k


def test_told_fitness_is_consumed_before_the_call_returns(P):
    n, lam = 30, 24
    st = synth.random_state(n, lam, seed=4, gen=4)
    lib = P.library()
    with P.CMAES(n, lam, 1.0, seed=1, precision="fp64", eigen_interval=2) as es:
        es.set_state(st)
        X = es.ask()
        f = np.ascontiguousarray(O.rot_ellipsoid(X))
        fc = f.copy()
        rc = lib.cmaes_tell(es.h, fc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        fc[:] = np.nan
        assert rc == 0, P.cmaes_last_error()
        g = es.state()
    o = oracle_state(st, kappa=2)
    Z = np.linalg.solve(np.diag(st["D"]), st["B"].T @ ((X - st["m"][:, None]) / st["sigma"]))
    O.generation(o, None, Z=Z, fvals=f)
    assert rel(g["m"], o.m) < 1e-10 and rel(g["C"], o.C) < 1e-10


def test_stopped_descent_refuses_generations(P):
    n, lam = 12, 10
    lib = P.library()
    with P.CMAES(n, lam, 2.0, seed=3, precision="fp64", objective="sphere", max_gens=2) as es:
        es.generation()
        es.generation()            # MaxGen fires at generation 2
        s = es.state(arrays=False)
        assert "maxgen" in s["stop_names"]
        assert lib.cmaes_generation(es.h) == P.binding.CMAES_ESTATE
        X = np.zeros((n, lam), order="F")
        assert lib.cmaes_ask(es.h, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == P.binding.CMAES_ESTATE
        assert es.state(arrays=False)["gen"] == 2      # nothing was queued
        # a restart clears the stop
        assert es.restart_ipop() == 0
        es.generation()
        assert es.state(arrays=False)["gen"] == 1
        es.generation()
        assert lib.cmaes_generation(es.h) == P.binding.CMAES_ESTATE
        # so does set_state
        full = es.state()
        es.set_state({"n": n, "lambda": full["lambda"], "gen": 0, "sigma": full["sigma"]})
        assert lib.cmaes_generation(es.h) == 0


def test_non_finite_covariance_returns_enumeric(P):
    n, lam = 40, 64
    R, xs = synth.problem(n, seed=2)
    lib = P.library()
    with P.CMAES(n, lam, 2.0, seed=2, precision="mixed", objective="rastrigin", R=R, xstar=xs,
                 eigen_interval=1) as es:
        for _ in range(3):
            es.generation()
        s = es.state()
        C = s["C"].copy()
        C[1, 7] = C[7, 1] = np.inf
        C[7, 7] = np.inf           # a non-finite diagonal entry also raises NUMERIC
        es.set_state({"n": n, "lambda": lam, "gen": s["gen"], "sigma": s["sigma"], "C": C})
        assert lib.cmaes_generation(es.h) == P.binding.CMAES_ENUMERIC
        st = es.state(arrays=False)
        assert "conditioncov" in st["stop_names"] and "numeric" in st["stop_names"], st["stop_names"]
        assert lib.cmaes_generation(es.h) == P.binding.CMAES_ESTATE
        assert es.restart_ipop() == 0
        es.generation()
        assert es.state(arrays=False)["stop"] == 0


def test_torch_allocator_hook(P):
    import torch
    n, lam = 64, 96
    R, xs = synth.problem(n, seed=5)
    outs = []
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    for alloc in (None, "torch"):
        with P.CMAES(n, lam, 2.0, seed=9, precision="mixed", objective="ellipsoid", R=R, xstar=xs,
                     eigen_interval=1, allocator=alloc) as es:
            for _ in range(4):
                es.generation()
            outs.append(es.state())
            used = torch.cuda.memory_allocated() - base
            if alloc == "torch":
                # C, B (n x n float64 each) at least came from torch's allocator
                assert used >= 2 * 8 * n * n, used
                assert len(es.allocator.live) > 10
                # the hook is fixed once the handle has allocated
                opt = P.cmaes_get_options(es.h)
                opt.dev_malloc = P.binding.DEV_MALLOC()
                opt.dev_free = P.binding.DEV_FREE()
                with pytest.raises(P.CmaesError) as e:
                    P.cmaes_set_options(es.h, opt)
                assert e.value.code == P.binding.CMAES_ESTATE
            else:
                assert used == 0
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base      # every block went back
    for k in ("m", "C", "B", "D", "p_sigma", "p_c", "f"):
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_allocator_hook_needs_both_functions(P):
    with P.CMAES(8, 8, 1.0, seed=1) as es:
        opt = P.cmaes_get_options(es.h)
        alloc = P.binding.TorchAllocator()
        opt.dev_malloc = alloc.c_malloc
        with pytest.raises(P.CmaesError) as e:
            P.cmaes_set_options(es.h, opt)
        assert e.value.code == P.binding.CMAES_EINVAL
