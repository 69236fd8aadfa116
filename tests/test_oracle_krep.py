"""Pins of the oracle's K-Replicated strategy (Alg. 3): with one leaf it is
a plain descent with the leaf's seed; while the leaves run, every lockstep
generation costs k_max * lambda_start evaluations; a parent starts only after
both children stopped, with twice their population."""

import oracle as O


def test_single_leaf_is_a_plain_descent():
    obj = O.Objective("sphere")
    best, evals, gens, log = O.k_replicated(6, 8, 1, 1.5, 7, obj)
    st = O.new_descent(6, 8, 1.5, O.krep_leaf_seed(7, 0))
    while not st.stop:
        O.generation(st, obj)
    assert best == st.f_best and evals == st.evals and gens == st.gen


def test_tree_mechanics():
    obj = O.Objective("sphere")
    so = O.StopOptions(max_gens=5, f_target=-1.0)        # every descent stops after 5 generations
    best, evals, gens, log = O.k_replicated(4, 6, 4, 1.0, 3, obj, so=so)
    # 3 levels of 5 generations each; the level-l descents run 4 >> l at a time with 6 * 2^l points
    assert gens == 15
    assert evals == 3 * 5 * 4 * 6
    lams = [rec["lam"] for rec in log]
    assert lams == [6] * 4 + [12] * 2 + [24]
    assert all(rec["gens"] == 5 for rec in log)


def test_leaf_seeds_are_distinct():
    seeds = {O.krep_leaf_seed(1, j) for j in range(1024)}
    assert len(seeds) == 1024 and all(0 <= s < 2 ** 64 for s in seeds)
