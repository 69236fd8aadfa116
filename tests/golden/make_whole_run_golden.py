"""Writes whole_runs.json: whole IPOP-CMA-ES runs of the FP64 oracle (Alg. 2,
Sec. 2.2) on the synthetic stand-ins of the paper's Sec. 4.1 workloads, the
expected values of the GPU whole-run tests.  Calls only oracle/ and synth/.

* config 1: plain CMA-ES, sphere, n = 10, lambda = 10, eigendecomposition
  every generation, stop at f < 1e-8 or 2000 generations; seeds 1..15.
* config 2: IPOP-CMA-ES, rotated ellipsoid (condition 1e6) with R Haar and
  x* uniform in [-4, 4]^n from synth.problem(100, seed), n = 100,
  lambda_start = 17 doubling up to K_max = 2^9, sigma0 = 2; seeds 1..15.
* config 5, scaled down: one descent on the rotated ellipsoid (condition
  1e6) at n = 100 with lambda = 2n = 200 and mu = lambda / 2 -- the large
  workload's ratios (n = 2000, lambda = 4096, mu = 2048) at a size the oracle
  finishes whole runs of; automatic eigendecomposition interval; sigma0 = 2;
  stop at f < 1e-8 or 20000 generations; seeds 1..15.  The GPU runs it with
  bf16x3 sampling.

Run: python tests/golden/make_whole_run_golden.py [config ...]  (all: about
ten minutes; named configs are recomputed and merged into the existing file)
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import synth  # noqa: E402

SEEDS = list(range(1, 16))


def config1(seed):
    st = O.new_descent(10, 10, 2.0, seed, kappa=1)
    so = O.StopOptions(max_gens=2000)
    while not st.stop:
        O.generation(st, O.Objective("sphere"), so=so)
    return {"seed": seed, "evals": st.evals, "gens": st.gen, "f_best": st.f_best, "stop": st.stop}


def config2(seed):
    n = 100
    R, xs = synth.problem(n, seed)
    best, _, log = O.ipop(n, 17, 2.0, seed, O.Objective("ellipsoid", R, xs), k_max=2 ** 9)
    return {"seed": seed, "evals": int(sum(d["evals"] for d in log)), "descents": len(log),
            "gens": [d["gens"] for d in log], "f_best": best}


CONFIG5_N, CONFIG5_LAMBDA = 100, 200


def config5(seed):
    n = CONFIG5_N
    R, xs = synth.problem(n, seed)
    st = O.new_descent(n, CONFIG5_LAMBDA, 2.0, seed)
    so = O.StopOptions(max_gens=20000)
    while not st.stop:
        O.generation(st, O.Objective("ellipsoid", R, xs), so=so)
    return {"seed": seed, "evals": st.evals, "gens": st.gen, "f_best": st.f_best, "stop": st.stop,
            "kappa": st.p.kappa}


CONFIGS = {"config1": config1, "config2": config2, "config5": config5}


def main(names):
    path = os.path.join(HERE, "whole_runs.json")
    out = {"source": "oracle/cmaes_oracle.py via tests/golden/make_whole_run_golden.py",
           "cite": "Alg. 2 (IPOP restarts, Sec. 2.2); Sec. 4.1 set-up (sigma0 = a quarter of the box)"}
    if names and os.path.exists(path):
        with open(path) as fh:
            out = json.load(fh)
    for name in names or list(CONFIGS):
        fn = CONFIGS[name]
        t0 = time.time()
        runs = [fn(s) for s in SEEDS]
        out[name] = runs
        print(name, f"{time.time() - t0:.1f}s", [r["evals"] for r in runs], flush=True)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
