"""Throughput of one IPOP-CMA-ES generation on one MI355X.

A step is one full generation (sample -> fused fitness -> rank -> recombine ->
paths/sigma -> rank-one + rank-mu covariance update -> eigendecomposition ->
stop tests) of the K = 2^8 descent of the headline workload: n = 1000,
lambda = 6144, rotated Rastrigin, mixed precision (float32 MFMA sampling,
fitness and SYRK; float64 eigensolve, paths and sigma).  Inputs are seeded and
synthetic and resident in HBM before timing starts.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma_tflops": 157.3, "fp64_tflops": 78.6, "bf16_mfma_tflops": 2500.0, "hbm_gbs": 8000.0}


def jacobi_round_work(n):
    """Work of one block-Jacobi round launch at dimension n (padded N, 16-index
    blocks, N/16 - 1 rounds per sweep).

    flops: the algorithmic count of a cyclic Jacobi sweep's two-sided update
    of A, 6 n^3 (each of the n(n-1)/2 rotations updates two rows and two
    columns, 6 flops per entry pair), spread over the sweep's rounds -- the
    unit in which the float64 eigensolve is priced against the float64 peak.
    executed_flops: what one round's float64 MFMA products execute (the
    lower 32 x 32 tiles Q1^T X Q2 of A and the 32-column pieces V Q of V).
    bytes: the lower block-pair tiles of A in, all of A out, all of V in and
    out (float64)."""
    N = 32 * ((n + 31) // 32)
    q = N // 32                      # block pairs per round
    rounds = N // 16 - 1
    flops = 6.0 * n ** 3 / rounds
    executed = 2 * (2.0 * 32 ** 3) * (q * (q + 1) // 2) + 2.0 * 32 * 32 * N * q
    nbytes = 8.0 * ((q * (q + 1) // 2) * 32 * 32 + 3 * N * N)
    return {"flops": flops, "executed_flops": executed, "bytes": nbytes, "rounds_per_sweep": rounds}


def kernel_work(n, lam, precision, sweeps, syrk_cfg=None):
    """Algorithmic work per launch of each timed kernel: (amount, unit, peak,
    bound)."""
    mu = lam // 2
    f32 = precision != "fp64"
    mm = PEAK["fp32_mfma_tflops"] if f32 else PEAK["fp64_tflops"]
    esz = 4 if f32 else 8
    # the Jacobi round runs its tile and V updates on the float64 matrix
    # cores; it is priced in float64 flops against the float64 peak (its
    # bytes, ~4.7 flop/B, stay within the caches' reach, and its time is set
    # by the chain of dependent pair-solve steps)
    jac = jacobi_round_work(n)["flops"]
    # the mixed covariance epilogue reads each split's float32 partial of every
    # lower 32 x 32 block (4 KiB), the lower triangle of C, and writes all of C
    epi = None
    if f32 and syrk_cfg is not None:
        import paper_2409_11765_amd as P
        _, _, splits = P.cmaes_syrk_plan(syrk_cfg, n, mu)
        nb = (n + 31) // 32
        epi = 4096.0 * splits * (nb * (nb + 1) // 2) + 8.0 * (n * (n + 1) // 2 + n * n)
    work = {
        "normals": (esz * n * lam, "GB/s", PEAK["hbm_gbs"], "hbm"),
        "sample_gemm": (2.0 * n * n * lam, "TFLOP/s", mm, "mfma"),
        "fitness": (2.0 * n * n * lam, "TFLOP/s", mm, "mfma"),
        "syrk": (float(n) * (n + 1) * mu, "TFLOP/s", mm, "mfma"),
        "eig_gemm": (2.0 * n ** 3, "TFLOP/s", PEAK["fp64_tflops"], "mfma"),
        "jacobi": (jac, "TFLOP/s", PEAK["fp64_tflops"], "mfma"),
        "rank": (float(lam) * lam, "Gcmp/s", None, "alu"),
    }
    if epi is not None:
        work["syrk_epi"] = (epi, "GB/s", PEAK["hbm_gbs"], "hbm")
    return work


def roofline_entry(name, kt, work):
    amount, unit, peak, bound = work[name]
    avg = kt[name]["avg_us"]
    if not avg:
        return None
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    achieved = amount / (avg * 1e-6) / scale
    return {"kernel": name, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak if peak else None, "avg_launch_us": avg,
            "launches_per_step": kt[name]["calls"], "work_per_launch": amount}
def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/traffic.json), or None when absent or when the kernel's
    source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        entry = json.load(fh).get(kernel)
    if not entry:
        return None
    with open(os.path.join(ROOT, entry["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != entry["source_sha256"]:
            return None
    return entry["hbm_bytes_per_launch"]


METRIC = "evals/s + gens/s at n=1000, λ=6144 (mixed vs FP64); % of MFMA/HBM peak"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--lam", type=int, default=6144)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="timed generations of the float64 path (default: --steps, on the same window)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=10,
                    help="generations of the concurrent-restart batch (10 descents, n=200); 0 = skip")
    ap.add_argument("--no-tune", action="store_true", help="keep the default float32 GEMM tiles")
    ap.add_argument("--calib", action="store_true",
                    help="first run a plain in-place negation of 256 MiB three times (a copy kernel of known "
                         "traffic, for scaling HBM counters)")
    ap.add_argument("--ablation", action="store_true",
                    help="instead of the headline line: per-phase mixed-vs-FP64 table over n and K")
    ap.add_argument("--large", action="store_true",
                    help="instead of the headline line: the large workload (n=2000, lambda=4096, rotated "
                         "ellipsoid, bf16x3 sampling)")
    ap.add_argument("--large-steps", type=int, default=50)
    ap.add_argument("--no-large", action="store_true",
                    help="leave the large workload (n=2000, lambda=4096) out of the headline line")
    ap.add_argument("--ert", action="store_true",
                    help="instead of the headline line: ERT / ECDF of IPOP, K-Distributed and K-Replicated on "
                         "synthetic functions")
    ap.add_argument("--asktell", action="store_true",
                    help="instead of the headline line: host ask/tell throughput with added evaluation cost")
    ap.add_argument("--tiles", default=None, help="force tiles: sample,fitness,syrk configuration indices")
    return ap.parse_args()


def run_gpu(P, torch, n, lam, precision, steps, warmup, seed, R, xs, tune=True, tiles=None, objective="rastrigin"):
    # a dedicated (default-priority) torch stream, handed to the library, so
    # the timing events below bracket exactly the library's work
    stream = torch.cuda.Stream()
    es = P.CMAES(n, lam, 2.0, seed=seed, precision=precision, objective=objective, R=R, xstar=xs,
                 stream=stream.cuda_stream)
    tiles_out = None
    try:
        if precision != "fp64":
            # the float32 GEMM tiles for this shape (untimed set-up)
            if tiles is not None:
                for site, cfg in zip(P.SITES, tiles):
                    es.set_gemm_config(site, cfg)
            elif tune:
                es.autotune(reps=10)
            tiles_out = {site: {"config": es.gemm_config(site),
                                "tile": P.cmaes_gemm_config_info(es.gemm_config(site))} for site in P.SITES}
            if hasattr(es, "last_tune_us"):
                tiles_out["tune_us"] = {site: [round(float(v), 2) for v in row]
                                        for site, row in zip(P.SITES, es.last_tune_us)}
        for _ in range(warmup):
            es.generation()
        torch.cuda.synchronize()
        # per-phase device times from the library's own HIP events (one extra generation)
        es.enable_timing(True)
        es.generation()
        phases = es.phase_times()
        es.enable_timing(False)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record(stream)
        for _ in range(steps):
            es.generation()
        t1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms = t0.elapsed_time(t1) / steps
        st = es.state(arrays=False)
        # per-kernel device time, on the handle's stream, in a separate pass:
        # the float32 tiles and the Jacobi rounds record their own dispatch
        # timestamps, the other kernels are bracketed by HIP events (which
        # add a little overhead to the generation)
        ksteps = max(2, min(steps, 5))
        es.enable_kernel_timing(True)
        for _ in range(ksteps):
            es.generation()
        torch.cuda.synchronize()
        kt = es.kernel_times()
        es.enable_kernel_timing(False)
        for v in kt.values():
            v["calls"] = v["calls"] / ksteps
            v["total_us"] = v["total_us"] / ksteps
    finally:
        es.close()
    return {"ms_per_step": ms, "wall_ms_per_step": 1e3 * wall / steps, "phases_us": phases, "state": st,
            "kernels": kt, "tiles": tiles_out}


def run_large(P, torch, steps, seed):
    """The large workload: n = 2000, lambda = 4096, mu = 2048, rotated
    ellipsoid (condition 1e6), y = B D z as bf16 hi/lo split products with
    float32 accumulation, float32 SYRK, float64 eigensolve every generation
    (the rule max(1, ceil(1/(10 n (c1 + cmu)))) gives 1 here)."""
    import synth
    n, lam = 2000, 4096
    R, xs = synth.problem(n, seed)
    res = run_gpu(P, torch, n, lam, "mixed_bf16x3", steps, 5, seed, R, xs, objective="ellipsoid")
    kt = res["kernels"]
    work = kernel_work(n, lam, "mixed", res["state"]["eig_sweeps"],
                       res["tiles"]["syrk"]["config"] if res["tiles"] else None)
    # the sampling product runs as three bf16 products: priced as executed
    # bf16 flops against the bf16 MFMA peak
    work["sample_gemm"] = (3 * 2.0 * n * n * lam, "TFLOP/s", PEAK["bf16_mfma_tflops"], "mfma")
    per_kernel = {k: roofline_entry(k, kt, work) for k in kt if kt[k]["calls"] and k in work}
    return {"workload": f"rotated ellipsoid (cond 1e6) n={n} lambda={lam} mu={lam // 2}, bf16x3 sampling, "
                        "float32 SYRK, float64 eigensolve every generation",
            "evals_per_s": lam * 1e3 / res["ms_per_step"], "gens_per_s": 1e3 / res["ms_per_step"],
            "ms_per_step": res["ms_per_step"], "steps": steps, "eig_sweeps_last": res["state"]["eig_sweeps"],
            "eig_corrections_last": res["state"]["eig_corrections"],
            "phases_us": res["phases_us"], "gemm_tiles": res["tiles"],
            "kernels": {k: {**kt[k], "roofline": per_kernel.get(k)} for k in kt}}


def run_batch(P, torch, steps, warmup, seed):
    """Concurrent restarts: 10 descents, n = 200, lambda_k = 19 * 2^k, rotated
    Rastrigin, mixed precision; one batch generation advances every descent."""
    import synth
    K, n = 10, 200
    lams = [19 * 2 ** k for k in range(K)]
    seeds = [seed * 100 + k for k in range(K)]
    with P.CMAESBatch([n] * K, lams, [2.0] * K, seeds, precision="mixed") as b:
        for k in range(K):
            R, xs = synth.problem(n, seeds[k])
            b.set_objective(k, "rastrigin", R, xs)
        for _ in range(warmup):
            b.generation()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.generation()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    return {"workload": "10 concurrent descents, n=200, lambda_k=19*2^k (k=0..9), rotated Rastrigin, mixed",
            "evals_per_s": sum(lams) * steps / el, "batch_gens_per_s": steps / el,
            "ms_per_batch_generation": 1e3 * el / steps, "sum_lambda": sum(lams)}


def rel_err(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / (nb if nb > 0 else 1.0)


def cpu_baseline(P, n, lam, seed, R, xs, budget_s, precisions=("mixed", "fp64")):
    """The FP64 oracle timed on the host, and each device path's error against
    it at the same shape.

    The oracle runs generations of the workload from a seeded synthetic
    descent state (eigenvalues log-spaced over two decades, sigma = 0.5) for
    about budget_s seconds; the first of them uses a seeded injected z.  The
    device paths run that same first generation (same state, same z) through
    cmaes_generation_with_z, and their results are compared with the
    oracle's: normwise m, sigma, C, p_sigma, p_c, the fitness values element
    by element, the eigenvalues, and the device's own reconstruction
    C = B D^2 B^T and orthogonality."""
    import oracle as O
    import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:
        threads = 1
    st = synth.random_state(n, lam, seed=seed + 100, cond=100.0, sigma=0.5, gen=20)
    Z = synth.normal_matrix(n, lam, seed=seed + 200)
    dev = {}
    for prec in precisions:
        with P.CMAES(n, lam, 2.0, seed=seed, precision=prec, objective="rastrigin", R=R, xstar=xs) as es:
            es.set_state(st)
            es.generation_with_z(Z)
            dev[prec] = es.state()
    o = O.new_descent(n, lam, 2.0, seed)
    o.m, o.sigma, o.C, o.B, o.D = st["m"].copy(), st["sigma"], st["C"].copy(), st["B"].copy(), st["D"].copy()
    o.ps, o.pc, o.gen = st["p_sigma"].copy(), st["p_c"].copy(), st["gen"]
    obj = O.Objective("rastrigin", R, xs)
    gens, t0 = 0, time.perf_counter()
    info = O.generation(o, obj, Z=Z)
    gens += 1
    ref = {"m": o.m.copy(), "sigma": o.sigma, "C": o.C.copy(), "p_sigma": o.ps.copy(), "p_c": o.pc.copy(),
           "D": o.D.copy(), "f": info["f"].copy()}
    while True:
        el = time.perf_counter() - t0
        if el >= budget_s or el / gens * (gens + 1) > 2.0 * budget_s:
            break
        O.generation(o, obj)
        gens += 1
    el = time.perf_counter() - t0
    errors = {}
    for prec, g in dev.items():
        Cg, Bg, Dg = g["C"], g["B"], g["D"]
        errors[prec] = {
            "m": rel_err(g["m"], ref["m"]), "sigma": abs(g["sigma"] - ref["sigma"]) / ref["sigma"],
            "C": rel_err(Cg, ref["C"]), "p_sigma": rel_err(g["p_sigma"], ref["p_sigma"]),
            "p_c": rel_err(g["p_c"], ref["p_c"]),
            "f_max_rel": float(np.max(np.abs(g["f"] - ref["f"]) / np.abs(ref["f"]))),
            "eigenvalues_max_rel": float(np.max(np.abs(Dg ** 2 - ref["D"] ** 2)) / np.max(ref["D"] ** 2)),
            "reconstruction": rel_err((Bg * Dg ** 2) @ Bg.T, Cg),
            "orthogonality": float(np.max(np.abs(Bg.T @ Bg - np.eye(n)))),
        }
    return {"value": lam * gens / el, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{gens} FP64 oracle generation(s) of the n={n}, lambda={lam} rotated-Rastrigin workload "
                      f"from a seeded synthetic descent state ({el:.1f} s, NumPy/OpenBLAS {threads} threads, "
                      f"eigendecomposition every generation)",
            "gens_per_s": gens / el, "oracle_error": errors}


def default_lambda(n):
    return 4 + int(np.floor(3.0 * np.log(n)))


def run_ablation(P, torch, seed, gens=9, warmup=2):
    """Per-phase device time, mixed vs FP64, for n in {10, 40, 200, 1000} and
    K in {1, 2^8} (lambda = K * default lambda), rotated Rastrigin."""
    import synth
    rows = []
    for n in (10, 40, 200, 1000):
        R, xs = synth.problem(n, seed)
        for K in (1, 256):
            lam = K * default_lambda(n)
            row = {"n": n, "K": K, "lambda": lam}
            for prec in ("fp64", "mixed"):
                stream = torch.cuda.Stream()
                with P.CMAES(n, lam, 2.0, seed=seed, precision=prec, objective="rastrigin", R=R, xstar=xs,
                             stream=stream.cuda_stream) as es:
                    if prec != "fp64":
                        es.autotune(reps=3)
                    for _ in range(warmup):
                        es.generation()
                    es.enable_timing(True)
                    acc = {k: 0.0 for k in P.PHASES}
                    for _ in range(gens):
                        es.generation()
                        for k, v in es.phase_times().items():
                            acc[k] += v / gens
                    es.enable_timing(False)
                    es.enable_graphs(True)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(gens):
                        es.generation()
                    torch.cuda.synchronize()
                    wall = (time.perf_counter() - t0) / gens
                row[prec] = {"phases_us": {k: round(v, 1) for k, v in acc.items()},
                             "device_us": round(sum(acc.values()), 1), "wall_us": round(1e6 * wall, 1)}
            row["mixed_speedup"] = {k: (row["fp64"]["phases_us"][k] / row["mixed"]["phases_us"][k]
                                        if row["mixed"]["phases_us"][k] > 0 else None) for k in P.PHASES}
            row["mixed_speedup_total"] = row["fp64"]["wall_us"] / row["mixed"]["wall_us"]
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    return rows


def run_asktell(P, torch, seed, n=200, lam=4864, gens=6, delays_ms=(0, 1, 10, 100)):
    """Host blackbox path: ask -> (host evaluation + added delay) -> tell, the
    paper's granularity axis (each generation's lambda evaluations run in
    parallel and cost the added delay once).  Serial: one descent.
    Overlapped: two descents in two host threads, so the device update of one
    overlaps the host evaluation of the other."""
    import threading
    import synth
    xs = synth.optimum(n, seed)

    def evaluate(X, delay):
        # shifted sphere on the host (the blackbox), plus the added cost
        D = X - xs[:, None]
        f = np.einsum("ij,ij->j", D, D)
        if delay > 0:
            time.sleep(delay)
        return f

    def descent(es, delay, count, out, idx):
        t0 = time.perf_counter()
        for _ in range(count):
            X = es.ask()
            es.tell(evaluate(X, delay))
        out[idx] = time.perf_counter() - t0

    res = []
    for d in delays_ms:
        delay = d / 1000.0
        handles = [P.CMAES(n, lam, 2.0, seed=seed + i, precision="mixed") for i in range(2)]
        try:
            for es in handles:
                es.autotune(reps=3)
                X = es.ask()
                es.tell(evaluate(X, 0.0))
            out = [0.0, 0.0]
            descent(handles[0], delay, gens, out, 0)
            serial = gens / out[0]
            ths = [threading.Thread(target=descent, args=(handles[i], delay, gens, out, i)) for i in range(2)]
            t0 = time.perf_counter()
            for t in ths:
                t.start()
            for t in ths:
                t.join()
            both = 2 * gens / (time.perf_counter() - t0)
        finally:
            for es in handles:
                es.close()
        res.append({"delay_ms": d, "serial_gens_per_s": serial, "serial_evals_per_s": serial * lam,
                    "two_descents_gens_per_s": both, "two_descents_evals_per_s": both * lam,
                    "overlap_gain": both / serial})
        print(json.dumps(res[-1]), file=sys.stderr, flush=True)
    return {"workload": f"n={n}, lambda={lam} (K=2^8), mixed; host-side shifted sphere (NumPy) + added delay "
                        f"per generation", "rows": res}


TARGETS = [1e2, 10 ** 1.5, 1e1, 10 ** 0.5, 1e0, 1e-2, 1e-4, 1e-6, 1e-8]


def _trace_run(step, budget_s):
    """Run `step()` (one lockstep generation, returning (total_evals, f_best,
    finished)) until finished, the last target is hit or the budget is spent;
    return the first (seconds, evals) at which each target was hit, and the
    run's total (seconds, evals)."""
    hits = [None] * len(TARGETS)
    t0 = time.perf_counter()
    evals, el = 0, 0.0
    while True:
        evals, fbest, finished = step()
        el = time.perf_counter() - t0
        for i, tg in enumerate(TARGETS):
            if hits[i] is None and fbest <= tg:
                hits[i] = (el, evals)
        if finished or hits[-1] is not None or el > budget_s:
            return hits, (el, evals)


def run_ert(P, torch, seeds=(1, 2, 3), dims=(10, 40), budget_s=3.0, kmax=64, lam0=12):
    """ERT and ECDF over the paper's nine targets (Sec. 4.3.1) for sequential
    IPOP-CMA-ES, K-Distributed (one descent per K = 1..K_max, restart on
    finish) and K-Replicated (Alg. 3), on the synthetic functions; f* = 0, so
    the quality is the best f found.  Time is wall-clock seconds on one GPU."""
    import synth
    funcs = ["sphere", "ellipsoid", "rastrigin"]
    levels = int(np.log2(kmax)) + 1
    rows, ecdf_pts = [], {}
    for n in dims:
        for fn in funcs:
            per_algo = {"ipop": [], "kdist": [], "krep": []}
            for seed in seeds:
                R, xs = synth.problem(n, seed)
                Rm = None if fn == "sphere" else R
                # sequential IPOP: lambda doubles at every stop until K_max
                es = P.CMAES(n, lam0, 2.0, seed=seed, precision="mixed", objective=fn, R=Rm, xstar=xs,
                             k_max=kmax)

                def step_ipop():
                    es.generation()
                    st = es.state(arrays=False)
                    done = False
                    if st["stop"] and not st["f_best"] <= TARGETS[-1]:
                        try:
                            es.restart_ipop()
                        except P.CmaesError:
                            done = True
                    return st["total_evals"], st["f_best"], done or st["f_best"] <= TARGETS[-1]
                per_algo["ipop"].append(_trace_run(step_ipop, budget_s))
                es.close()
                # K-Distributed: all K at once, each restarting with its own lambda
                b = P.CMAESBatch([n] * levels, [lam0 * 2 ** k for k in range(levels)], [2.0] * levels,
                                 [seed * 100 + k for k in range(levels)], precision="mixed")
                for k in range(levels):
                    b.set_objective(k, fn, Rm, xs)

                def step_kdist():
                    b.generation()
                    fbest, _ = b.best()
                    ev = sum(b.state(k, arrays=False)["total_evals"] for k in range(levels))
                    return ev, fbest, fbest <= TARGETS[-1]
                per_algo["kdist"].append(_trace_run(step_kdist, budget_s))
                b.close()
                # K-Replicated: binary tree of descents over kmax * lam0 slots
                r = P.KReplicated(n, lam0, kmax, 2.0, seed=seed, precision="mixed", objective=fn, R=Rm, xstar=xs)

                def step_krep():
                    r.generation()
                    st = r.status()
                    return st["total_evals"], st["f_best"], bool(st["done"])
                per_algo["krep"].append(_trace_run(step_krep, budget_s))
                r.close()
            for algo, runs in per_algo.items():
                for i, tg in enumerate(TARGETS):
                    succ = [h[i] for h, _ in runs if h[i] is not None]
                    tot_s = sum((h[i][0] if h[i] is not None else tot[0]) for h, tot in runs)
                    tot_e = sum((h[i][1] if h[i] is not None else tot[1]) for h, tot in runs)
                    rows.append({"n": n, "f": fn, "algo": algo, "target": tg, "successes": len(succ),
                                 "runs": len(runs), "ert_s": tot_s / len(succ) if succ else None,
                                 "ert_evals": tot_e / len(succ) if succ else None})
                ecdf_pts.setdefault((n, algo), []).extend(
                    h[i][0] if h[i] is not None else float("inf") for h, _ in runs for i in range(len(TARGETS)))
            print(json.dumps({"n": n, "f": fn, "done": True}), file=sys.stderr, flush=True)
    grid = [0.003, 0.01, 0.03, 0.1, 0.3, 1.0, budget_s]
    ecdf = [{"n": n, "algo": algo, "t_s": grid,
             "fraction": [float(np.mean(np.asarray(v) <= t)) for t in grid]} for (n, algo), v in ecdf_pts.items()]
    return {"targets": TARGETS, "seeds": list(seeds), "budget_s": budget_s, "k_max": kmax, "lambda_start": lam0,
            "ert": rows, "ecdf": ecdf}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import paper_2409_11765_amd as P
    import synth

    n, lam = a.n, a.lam
    R, xs = synth.problem(n, a.seed)
    torch.cuda.set_device(0)
    if a.calib:
        x = torch.empty(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        x.fill_(1.0)
        for _ in range(3):
            x.neg_()
        torch.cuda.synchronize()
    if a.ablation:
        print(json.dumps({"ablation": run_ablation(P, torch, a.seed)}), flush=True)
        return
    if a.asktell:
        print(json.dumps({"asktell": run_asktell(P, torch, a.seed)}), flush=True)
        return
    if a.ert:
        print(json.dumps({"ert": run_ert(P, torch)}), flush=True)
        return
    if a.large:
        print(json.dumps({"large": run_large(P, torch, a.large_steps, a.seed)}), flush=True)
        return
    tiles = [int(v) for v in a.tiles.split(",")] if a.tiles else None
    mixed = run_gpu(P, torch, n, lam, a.precision, a.steps, a.warmup, a.seed, R, xs, tune=not a.no_tune,
                    tiles=tiles)
    fp64 = None
    if not a.no_fp64:
        # the same warm-up and timed window of the descent as the mixed path
        fp64 = run_gpu(P, torch, n, lam, "fp64", a.fp64_steps or a.steps, a.warmup, a.seed, R, xs)
    gens = 1e3 / mixed["ms_per_step"]
    mu = lam // 2
    ph = mixed["phases_us"]
    flop_sample = 2.0 * n * n * lam
    flop_fit = 2.0 * n * n * lam
    flop_syrk = float(n) * (n + 1) * mu
    gemm_us = ph["sample"] + ph["fitness"] + ph["covariance"]
    frac = lambda fl, us: (fl / (us * 1e-6)) / 1e12 / PEAK["fp32_mfma_tflops"] if us > 0 else None
    # phase times come from one extra generation queued eagerly with an event
    # between phases (serialised, no graph replay): shares of that pass's sum
    phase_share = {k: v / sum(ph.values()) for k, v in ph.items()}
    dom = max(ph, key=ph.get)
    out = {
        "metric": METRIC,
        "value": lam * gens,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if a.precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": f"IPOP-CMA-ES K=2^8 descent, rotated Rastrigin n={n} lambda={lam} mu={mu}, "
                               f"{a.precision} precision, eigendecomposition every generation",
                   "n": n, "lambda": lam, "mu": mu, "precision": a.precision, "parallelism": "single GPU"},
        "gens_per_s": gens,
        "eig_sweeps_last": mixed["state"]["eig_sweeps"],
        "eig_corrections_last": mixed["state"]["eig_corrections"],
        "phases_us_eager": ph,
        "phase_share_eager": phase_share,
        "dominant_phase": dom,
        "gemm_mfma_frac": {"sample": frac(flop_sample, ph["sample"]), "fitness": frac(flop_fit, ph["fitness"]),
                           "syrk": frac(flop_syrk, ph["covariance"]),
                           "all_gemm": frac(flop_sample + flop_fit + flop_syrk, gemm_us)},
    }
    if fp64 is not None:
        out["fp64"] = {"ms_per_step": fp64["ms_per_step"], "evals_per_s": lam * 1e3 / fp64["ms_per_step"],
                       "gens_per_s": 1e3 / fp64["ms_per_step"], "phases_us": fp64["phases_us"]}
        out["mixed_over_fp64"] = fp64["ms_per_step"] / mixed["ms_per_step"]
    kt = mixed["kernels"]
    # the same fractions from the kernels' own dispatch-timed durations (the
    # phase figures above also hold the small kernels around each product)
    kus = {k: kt[k]["total_us"] / kt[k]["calls"] for k in ("sample_gemm", "fitness", "syrk")
           if k in kt and kt[k]["calls"]}
    if len(kus) == 3:
        out["gemm_kernel_frac"] = {
            "sample": frac(flop_sample, kus["sample_gemm"]), "fitness": frac(flop_fit, kus["fitness"]),
            "syrk": frac(flop_syrk, kus["syrk"]),
            "sampling_and_rank_mu": frac(flop_sample + flop_syrk, kus["sample_gemm"] + kus["syrk"]),
            "all_gemm": frac(flop_sample + flop_fit + flop_syrk, sum(kus.values()))}
    syrk_cfg = mixed["tiles"]["syrk"]["config"] if mixed["tiles"] else None
    work = kernel_work(n, lam, a.precision, mixed["state"]["eig_sweeps"], syrk_cfg)
    per_kernel = {k: roofline_entry(k, kt, work) for k in kt if kt[k]["calls"] and k in work}
    dom_k = max((k for k in kt if kt[k]["calls"]), key=lambda k: kt[k]["total_us"])
    roof = dict(per_kernel[dom_k])
    roof["traffic"] = measured_traffic(dom_k)
    roof["share_of_step"] = kt[dom_k]["total_us"] / (1e3 * mixed["ms_per_step"])
    if dom_k == "jacobi":
        jw = jacobi_round_work(n)
        roof["executed_flops_per_launch"] = jw["executed_flops"]
        roof["executed_tflops"] = jw["executed_flops"] / (roof["avg_launch_us"] * 1e-6) / 1e12
        roof["bytes_per_launch"] = jw["bytes"]
        roof["achieved_gbs"] = jw["bytes"] / (roof["avg_launch_us"] * 1e-6) / 1e9
        roof["limiter"] = ("latency: each round waits for the previous round's pair solves (a chain of "
                           "dependent rotation steps) and for the launch before it")
    out["roofline"] = roof
    out["kernels"] = {k: {**kt[k], "roofline": per_kernel.get(k)} for k in kt}
    out["gemm_tiles"] = mixed["tiles"]
    if a.batch_steps > 0:
        out["batch"] = run_batch(P, torch, a.batch_steps, 3, a.seed)
    if not a.no_large:
        out["large"] = run_large(P, torch, a.large_steps, a.seed)
    if not a.no_cpu_baseline:
        cb = cpu_baseline(P, n, lam, a.seed, R, xs, a.cpu_seconds)
        # each result's error against the FP64 oracle, one generation from the
        # same state and z at the headline shape
        out["oracle_error"] = cb.pop("oracle_error")
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
