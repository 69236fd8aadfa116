"""The stored whole-run values (tests/golden/whole_runs.json) are the
oracle's: re-running a few config-1 seeds reproduces them exactly, and the
file's shape is what the GPU whole-run tests expect."""

import json
import os

import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "whole_runs.json")


def test_config1_values_are_the_oracles():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    for rec in g["config1"][:3]:
        st = O.new_descent(10, 10, 2.0, rec["seed"], kappa=1)
        so = O.StopOptions(max_gens=2000)
        while not st.stop:
            O.generation(st, O.Objective("sphere"), so=so)
        assert st.evals == rec["evals"] and st.f_best == rec["f_best"]


def test_whole_run_records():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    for name in ("config1", "config2"):
        assert [r["seed"] for r in g[name]] == list(range(1, 16))
        assert all(r["f_best"] < 1e-8 for r in g[name])
    assert all(r["descents"] >= 1 for r in g["config2"])
