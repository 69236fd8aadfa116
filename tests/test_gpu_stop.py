"""Stop tests of the device (Sec. 2.2 reading) against the oracle's, one
generation from injected states built to trigger each criterion: the stop
bits after the generation must be identical, and the targeted bit set."""

import numpy as np
import pytest

import oracle as O
import synth
from helpers import oracle_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_11765_amd as P
    return P


CASES = [
    # name, state overrides, options, expected bit(s)
    ("plain", {}, {}, 0),
    ("tolx_noeffect", {"sigma": 1e-20}, {}, O.STOP_TOLX | O.STOP_NOEFFECTAXIS | O.STOP_NOEFFECTCOORD),
    ("condition", {"cond": 1e16}, {}, O.STOP_CONDITIONCOV),
    ("maxgen", {}, {"max_gens": 4}, O.STOP_MAXGEN),
    ("ftarget", {}, {"f_target": 1e30}, O.STOP_FTARGET),
    ("numeric", {"m_nan": True}, {}, O.STOP_NUMERIC),
]


@pytest.mark.parametrize("name,over,opts,expect", CASES, ids=[c[0] for c in CASES])
def test_stop_bits_match_oracle(P, name, over, opts, expect):
    n, lam = 20, 12
    print(f"case stop {name}", flush=True)
    st = synth.random_state(n, lam, seed=41, cond=over.get("cond", 100.0), gen=3)
    if "sigma" in over:
        st["sigma"] = over["sigma"]
    if over.get("m_nan"):
        st["m"][5] = np.nan  # every f is NaN (ranked as +inf); m stays non-finite
    R, xs = synth.problem(n, seed=8)
    Z = synth.normal_matrix(n, lam, seed=19)
    es = P.CMAES(n, lam, 1.0, seed=1, precision="fp64", objective="rastrigin", R=R, xstar=xs, **opts)
    try:
        es.set_state(st)
        es.generation_with_z(Z)
        bits_dev = es.state(arrays=False)["stop"]
    finally:
        es.close()
    o = oracle_state(st)
    so = O.StopOptions(**opts)
    O.generation(o, O.Objective("rastrigin", R, xs), Z=Z, so=so)
    assert bits_dev == o.stop, (hex(bits_dev), hex(o.stop))
    if expect:
        assert bits_dev & expect == expect
    else:
        assert bits_dev == 0
