"""Graph replay of the fixed part of a generation (sampling through the
eigensolve set-up, captured once and replayed) against eager queueing of the
same launches: every generation's state must be bit-identical, across
replays of both captured variants (with and without an eigensolve), across an
IPOP restart that changes lambda and re-captures, with eager work (the
eigensolve sweeps, stop tests, state reads) between the replays."""

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


def _trajectory(P, n, lam, precision, gens, graphs, restart_at):
    R, xs = synth.problem(n, seed=n + 1)
    es = P.CMAES(n, lam, 2.0, seed=21, precision=precision, objective="rastrigin", R=R, xstar=xs)
    out = []
    try:
        es.enable_graphs(graphs)
        for g in range(gens):
            if g == restart_at:
                es.restart_ipop()
            es.generation()
            out.append(es.state())
    finally:
        es.close()
    return out


def _same(a, b):
    for k, v in a.items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, b[k], equal_nan=True), k
        else:
            assert v == b[k] or (v != v and b[k] != b[k]), k


@pytest.mark.parametrize("n,lam,precision", [(200, 19, "mixed"), (37, 53, "fp64"), (100, 17, "mixed_bf16x3"),
                                             (10, 10, "mixed")])
def test_graph_replay_bit_identical(P, n, lam, precision):
    print(f"case graph n={n} lam={lam} {precision}", flush=True)
    eager = _trajectory(P, n, lam, precision, 14, False, restart_at=7)
    graph = _trajectory(P, n, lam, precision, 14, True, restart_at=7)
    assert graph[-1]["lambda"] == 2 * lam
    for g, (a, b) in enumerate(zip(eager, graph)):
        _same(a, b)


def test_batch_graph_replay_bit_identical(P):
    n = [30, 30, 50]
    lam = [12, 24, 16]
    runs = []
    for graphs in (False, True):
        b = P.CMAESBatch(n, lam, [2.0] * 3, [5, 6, 7], precision="mixed")
        try:
            b.enable_graphs(graphs)
            for k in range(3):
                R, xs = synth.problem(n[k], seed=k + 3)
                b.set_objective(k, "rastrigin", R, xs)
            for _ in range(9):
                b.generation()
            runs.append([b.state(k) for k in range(3)])
        finally:
            b.close()
    for a, c in zip(*runs):
        _same(a, c)


def test_graph_off_with_timing(P):
    """Phase timing forces eager queueing; results do not depend on it."""
    n, lam = 64, 40
    R, xs = synth.problem(n, seed=2)
    st = []
    for timing in (False, True):
        es = P.CMAES(n, lam, 2.0, seed=3, precision="mixed", objective="ellipsoid", R=R, xstar=xs)
        try:
            es.enable_timing(timing)
            for _ in range(5):
                es.generation()
            st.append(es.state())
        finally:
            es.close()
    _same(st[0], st[1])
