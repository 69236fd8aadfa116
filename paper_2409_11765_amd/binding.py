"""ctypes binding of libcmaes_mi355x.so (the C ABI in include/cmaes_mi355x.h).

Argument marshalling only: every step of a generation runs in the library's
HIP kernels.  Functions keep the C names; failures raise ``CmaesError`` with
the library's message.  Host arrays are NumPy float64; matrices are passed in
column-major order (column k = candidate k), so ``X[:, k]`` is point k.

The library is loaded at import; a missing or unloadable library raises
ImportError (there is no fallback implementation).
"""

from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_PI32 = C.POINTER(C.c_int32)
_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcmaes_mi355x.so")

CMAES_OK, CMAES_EINVAL, CMAES_ENOMEM, CMAES_EDEVICE = 0, -1, -2, -3
CMAES_ESTATE, CMAES_EKMAX, CMAES_ENUMERIC = -4, -5, -6
CMAES_FP64, CMAES_MIXED, CMAES_MIXED_BF16X3 = 0, 1, 2
OBJECTIVES = {"none": 0, "sphere": 1, "ellipsoid": 2, "rastrigin": 3}
PRECISIONS = {"fp64": CMAES_FP64, "mixed": CMAES_MIXED, "mixed_bf16x3": CMAES_MIXED_BF16X3}
VARIANTS = {"standard": 0, "active": 1, "separable": 2}
STOP_BITS = ["tolhistfun", "tolfun", "tolx", "noeffectaxis", "noeffectcoord", "conditioncov",
             "ftarget", "maxgen", "maxevals", "numeric"]
NUM_PHASES = 6
KERNELS = ["normals", "sample_gemm", "fitness", "rank", "syrk", "eig_gemm", "jacobi", "syrk_epi"]
PHASES = ["sample", "fitness", "rank", "update", "covariance", "eigen"]


class CmaesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


DEV_MALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class CmaesOptions(C.Structure):
    _fields_ = [("precision", C.c_int32), ("eigen_interval", C.c_int32), ("k_max", C.c_int32),
                ("max_gens", C.c_int32), ("max_evals", C.c_int64), ("box_lo", C.c_double),
                ("box_hi", C.c_double), ("f_target", C.c_double), ("tol_hist_fun", C.c_double),
                ("tol_fun", C.c_double), ("tol_x_factor", C.c_double), ("max_condition", C.c_double),
                ("stream", C.c_void_p), ("dev_malloc", DEV_MALLOC), ("dev_free", DEV_FREE),
                ("alloc_ctx", C.c_void_p), ("variant", C.c_int32), ("reserved_", C.c_int32)]


class TorchAllocator:
    """The allocator hook of cmaes_options_t backed by PyTorch's caching
    allocator (device memory then shows up in torch.cuda.memory_allocated()).
    Blocks are associated with `stream` (the handle's stream when it is a torch
    stream, else torch's current stream); the library synchronises its own
    stream before it releases a block.  Keep the object alive as long as the
    handle (the CMAES wrapper does)."""

    def __init__(self, device=None, stream=None):
        import torch  # only this optional hook needs torch
        self._torch = torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = stream
        self.live = {}

        def _alloc(nbytes, _ctx):
            try:
                p = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:
                return None
            self.live[int(p)] = int(nbytes)
            return int(p)

        def _free(ptr, _ctx):
            if ptr:
                self.live.pop(int(ptr), None)
                self._torch.cuda.caching_allocator_delete(int(ptr))

        self.c_malloc = DEV_MALLOC(_alloc)
        self.c_free = DEV_FREE(_free)

    def install(self, opt: "CmaesOptions"):
        opt.dev_malloc = self.c_malloc
        opt.dev_free = self.c_free
        opt.alloc_ctx = None


_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)


class CmaesState(C.Structure):
    _fields_ = [("n", C.c_int32), ("lambda_", C.c_int32), ("mu", C.c_int32), ("restart", C.c_int32),
                ("gen", C.c_int64), ("evals", C.c_int64), ("total_evals", C.c_int64),
                ("sigma", C.c_double), ("f_best", C.c_double), ("stop", C.c_uint32), ("kappa", C.c_int32),
                ("eig_sweeps", C.c_int32), ("eig_corrections", C.c_int32), ("m", _PD), ("C", _PD), ("B", _PD), ("D", _PD), ("p_sigma", _PD), ("p_c", _PD),
                ("x_best", _PD), ("f", _PD), ("order", _PI)]


class KrepStatus(C.Structure):
    _fields_ = [("running", C.c_int32), ("finished", C.c_int32), ("lambda_max_running", C.c_int32),
                ("done", C.c_int32), ("lockstep_generations", C.c_int64), ("total_evals", C.c_int64),
                ("f_best", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    H = C.c_void_p
    sig = {
        "cmaes_default_options": (C.c_int, [C.POINTER(CmaesOptions)]),
        "cmaes_create": (H, [C.c_int, C.c_int, C.c_double, C.c_uint64]),
        "cmaes_destroy": (None, [H]),
        "cmaes_set_options": (C.c_int, [H, C.POINTER(CmaesOptions)]),
        "cmaes_get_options": (C.c_int, [H, C.POINTER(CmaesOptions)]),
        "cmaes_set_objective": (C.c_int, [H, C.c_int, _PD, _PD]),
        "cmaes_generation": (C.c_int, [H]),
        "cmaes_generation_with_z": (C.c_int, [H, _PD]),
        "cmaes_ask": (C.c_int, [H, _PD]),
        "cmaes_ask_noalloc": (C.c_int, [H, _PD]),
        "cmaes_tell": (C.c_int, [H, _PD]),
        "cmaes_restart_ipop": (C.c_int, [H]),
        "cmaes_ipop_run": (C.c_int, [H, C.POINTER(C.c_int)]),
        "cmaes_state": (C.c_int, [H, C.POINTER(CmaesState)]),
        "cmaes_set_state": (C.c_int, [H, C.POINTER(CmaesState)]),
        "cmaes_enable_timing": (C.c_int, [H, C.c_int]),
        "cmaes_phase_times": (C.c_int, [H, _PD]),
        "cmaes_enable_kernel_timing": (C.c_int, [H, C.c_int]),
        "cmaes_enable_graphs": (C.c_int, [H, C.c_int]),
        "cmaes_set_eigen_correction": (C.c_int, [H, C.c_int, C.c_double]),
        "cmaes_batch_enable_graphs": (C.c_int, [H, C.c_int]),
        "cmaes_kernel_times": (C.c_int, [H, _PD, C.POINTER(C.c_int64)]),
        "cmaes_last_error": (C.c_char_p, []),
        "cmaes_gemm_config_count": (C.c_int, []),
        "cmaes_gemm_config_info": (C.c_int, [C.c_int, _PI32, _PI32, _PI32]),
        "cmaes_set_gemm_config": (C.c_int, [H, C.c_int, C.c_int]),
        "cmaes_get_gemm_config": (C.c_int, [H, C.c_int, _PI32]),
        "cmaes_autotune": (C.c_int, [H, C.c_int, _PD, _PI32]),
        "cmaes_device_arch": (C.c_int, [C.c_char_p, C.c_int]),
        "cmaes_syrk_plan": (C.c_int, [C.c_int, C.c_int, C.c_int, _PI32, _PI32, _PI32]),
        "cmaes_batch_create": (H, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _PD, C.POINTER(C.c_uint64)]),
        "cmaes_batch_destroy": (None, [H]),
        "cmaes_batch_count": (C.c_int, [H]),
        "cmaes_batch_set_options": (C.c_int, [H, C.POINTER(CmaesOptions)]),
        "cmaes_batch_set_objective": (C.c_int, [H, C.c_int, C.c_int, _PD, _PD]),
        "cmaes_batch_generation": (C.c_int, [H]),
        "cmaes_batch_state": (C.c_int, [H, C.c_int, C.POINTER(CmaesState)]),
        "cmaes_batch_best": (C.c_int, [H, _PD, C.POINTER(C.c_int)]),
        "cmaes_krep_create": (H, [C.c_int, C.c_int, C.c_int, C.c_double, C.c_uint64]),
        "cmaes_krep_destroy": (None, [H]),
        "cmaes_krep_set_options": (C.c_int, [H, C.POINTER(CmaesOptions)]),
        "cmaes_krep_set_objective": (C.c_int, [H, C.c_int, _PD, _PD]),
        "cmaes_krep_generation": (C.c_int, [H]),
        "cmaes_krep_run": (C.c_int, [H, C.c_int64]),
        "cmaes_krep_status": (C.c_int, [H, C.POINTER(KrepStatus)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ["cmaes_default_options", "cmaes_create", "cmaes_destroy", "cmaes_set_options",
            "cmaes_get_options", "cmaes_set_objective", "cmaes_generation", "cmaes_generation_with_z",
            "cmaes_ask", "cmaes_ask_noalloc", "cmaes_tell", "cmaes_restart_ipop", "cmaes_ipop_run", "cmaes_state",
            "cmaes_set_state", "cmaes_enable_timing", "cmaes_phase_times", "cmaes_enable_kernel_timing",
            "cmaes_enable_graphs", "cmaes_batch_enable_graphs", "cmaes_set_eigen_correction",
            "cmaes_kernel_times", "cmaes_last_error", "cmaes_gemm_config_count", "cmaes_gemm_config_info",
            "cmaes_set_gemm_config", "cmaes_get_gemm_config", "cmaes_autotune", "cmaes_device_arch",
            "cmaes_syrk_plan", "cmaes_batch_create", "cmaes_batch_destroy",
            "cmaes_batch_count", "cmaes_batch_set_options", "cmaes_batch_set_objective", "cmaes_batch_generation",
            "cmaes_batch_state", "cmaes_batch_best", "cmaes_krep_create", "cmaes_krep_destroy",
            "cmaes_krep_set_options", "cmaes_krep_set_objective", "cmaes_krep_generation", "cmaes_krep_run",
            "cmaes_krep_status"]


def library():
    return _lib


def cmaes_last_error() -> str:
    return _lib.cmaes_last_error().decode()


def _check(rc, allow=()):
    if rc != CMAES_OK and rc not in allow:
        raise CmaesError(rc, cmaes_last_error())
    return rc


def _dptr(a):
    return a.ctypes.data_as(_PD) if a is not None else None


def _colmajor(a, shape):
    a = np.asarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return np.asfortranarray(a)


def cmaes_default_options() -> CmaesOptions:
    o = CmaesOptions()
    _check(_lib.cmaes_default_options(C.byref(o)))
    return o


def cmaes_create(n: int, lam: int, sigma0: float, seed: int):
    h = _lib.cmaes_create(int(n), int(lam), float(sigma0), int(seed) & 0xFFFFFFFFFFFFFFFF)
    if not h:
        raise CmaesError(CMAES_EINVAL, cmaes_last_error())
    return h


def cmaes_destroy(h):
    _lib.cmaes_destroy(h)


def cmaes_set_options(h, opt: CmaesOptions):
    _check(_lib.cmaes_set_options(h, C.byref(opt)))


def cmaes_get_options(h) -> CmaesOptions:
    o = CmaesOptions()
    _check(_lib.cmaes_get_options(h, C.byref(o)))
    return o


def cmaes_set_objective(h, kind, n: int, R=None, xstar=None):
    k = OBJECTIVES[kind] if isinstance(kind, str) else int(kind)
    Rf = _colmajor(R, (n, n)) if R is not None else None
    xs = np.ascontiguousarray(xstar, dtype=np.float64) if xstar is not None else None
    _check(_lib.cmaes_set_objective(h, k, _dptr(Rf), _dptr(xs)))


def cmaes_generation(h):
    _check(_lib.cmaes_generation(h))


def cmaes_generation_with_z(h, Z):
    # the library has copied Z when the call returns, so the temporary
    # column-major copy may be released right after
    Zf = np.asfortranarray(np.asarray(Z, dtype=np.float64))
    _check(_lib.cmaes_generation_with_z(h, _dptr(Zf)))


def cmaes_ask(h, n: int, lam: int) -> np.ndarray:
    X = np.empty((n, lam), dtype=np.float64, order="F")
    _check(_lib.cmaes_ask(h, _dptr(X)))
    return X


def cmaes_ask_noalloc(h, n: int, lam: int) -> np.ndarray:
    X = np.empty((n, lam), dtype=np.float64, order="F")
    _check(_lib.cmaes_ask_noalloc(h, _dptr(X)))
    return X


def cmaes_tell(h, f):
    fa = np.ascontiguousarray(f, dtype=np.float64)
    _check(_lib.cmaes_tell(h, _dptr(fa)))


def cmaes_restart_ipop(h) -> int:
    return _check(_lib.cmaes_restart_ipop(h), allow=(CMAES_EKMAX,))


def cmaes_ipop_run(h) -> int:
    d = C.c_int(0)
    _check(_lib.cmaes_ipop_run(h, C.byref(d)))
    return d.value


def cmaes_state(h, arrays: bool = True, _fetch=None) -> dict:
    fetch = _fetch or (lambda st: _lib.cmaes_state(h, C.byref(st)))
    s = CmaesState()
    _check(fetch(s))  # scalars first, to learn n and lambda
    out = {"n": s.n, "lambda": s.lambda_, "mu": s.mu, "restart": s.restart, "gen": s.gen,
           "evals": s.evals, "total_evals": s.total_evals, "sigma": s.sigma, "f_best": s.f_best,
           "stop": s.stop, "kappa": s.kappa, "eig_sweeps": s.eig_sweeps,
           "eig_corrections": s.eig_corrections}
    if arrays:
        n, lam = s.n, s.lambda_
        bufs = {k: np.zeros(n) for k in ("m", "D", "p_sigma", "p_c", "x_best")}
        bufs["C"] = np.zeros((n, n), order="F")
        bufs["B"] = np.zeros((n, n), order="F")
        bufs["f"] = np.zeros(lam)
        order = np.zeros(lam, dtype=np.int32)
        for k, v in bufs.items():
            setattr(s, k, _dptr(v))
        s.order = order.ctypes.data_as(_PI)
        _check(fetch(s))
        out.update(bufs)
        out["order"] = order
        out["sigma"], out["f_best"], out["stop"] = s.sigma, s.f_best, s.stop
    out["stop_names"] = [nm for i, nm in enumerate(STOP_BITS) if out["stop"] >> i & 1]
    return out


def cmaes_set_state(h, st: dict):
    s = CmaesState()
    s.n, s.lambda_ = int(st["n"]), int(st["lambda"])
    s.gen, s.sigma = int(st.get("gen", 0)), float(st["sigma"])
    keep = []
    n = s.n
    for k in ("m", "D", "p_sigma", "p_c"):
        if st.get(k) is not None:
            a = np.ascontiguousarray(st[k], dtype=np.float64)
            keep.append(a)
            setattr(s, k, _dptr(a))
    for k in ("C", "B"):
        if st.get(k) is not None:
            a = _colmajor(st[k], (n, n))
            keep.append(a)
            setattr(s, k, _dptr(a))
    _check(_lib.cmaes_set_state(h, C.byref(s)))


def cmaes_enable_timing(h, on: bool = True):
    _check(_lib.cmaes_enable_timing(h, 1 if on else 0))


def cmaes_phase_times(h) -> dict:
    out = np.zeros(NUM_PHASES)
    _check(_lib.cmaes_phase_times(h, _dptr(out)))
    return dict(zip(PHASES, out.tolist()))


def cmaes_enable_graphs(h, on: bool = True):
    _check(_lib.cmaes_enable_graphs(h, 1 if on else 0))


def cmaes_set_eigen_correction(h, on: bool = True, max_angle_norm: float = 2e-3):
    _check(_lib.cmaes_set_eigen_correction(h, 1 if on else 0, float(max_angle_norm)))


def cmaes_batch_enable_graphs(b, on: bool = True):
    _check(_lib.cmaes_batch_enable_graphs(b, 1 if on else 0))


def cmaes_enable_kernel_timing(h, on: bool = True):
    _check(_lib.cmaes_enable_kernel_timing(h, 1 if on else 0))


def cmaes_kernel_times(h) -> dict:
    tot = np.zeros(len(KERNELS))
    cnt = np.zeros(len(KERNELS), dtype=np.int64)
    _check(_lib.cmaes_kernel_times(h, _dptr(tot), cnt.ctypes.data_as(C.POINTER(C.c_int64))))
    return {k: {"total_us": float(t), "calls": int(c), "avg_us": float(t) / c if c else None}
            for k, t, c in zip(KERNELS, tot, cnt)}


SITES = ["sample", "fitness", "syrk"]


def cmaes_gemm_config_count() -> int:
    return int(_lib.cmaes_gemm_config_count())


def cmaes_gemm_config_info(cfg: int) -> tuple:
    v = [C.c_int32() for _ in range(3)]
    _check(_lib.cmaes_gemm_config_info(cfg, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def _site(site):
    return SITES.index(site) if isinstance(site, str) else int(site)


def cmaes_set_gemm_config(h, site, cfg: int):
    _check(_lib.cmaes_set_gemm_config(h, _site(site), int(cfg)))


def cmaes_get_gemm_config(h, site) -> int:
    v = C.c_int32()
    _check(_lib.cmaes_get_gemm_config(h, _site(site), C.byref(v)))
    return v.value


def cmaes_autotune(h, reps: int = 10):
    """Times every tile at each tunable site; returns (us[site][cfg], chosen[site])."""
    nc = cmaes_gemm_config_count()
    us = np.zeros(len(SITES) * nc)
    chosen = (C.c_int32 * len(SITES))()
    _check(_lib.cmaes_autotune(h, int(reps), _dptr(us), chosen))
    return us.reshape(len(SITES), nc), list(chosen)


def cmaes_device_arch() -> str:
    buf = C.create_string_buffer(128)
    _check(_lib.cmaes_device_arch(buf, len(buf)))
    return buf.value.decode()


def cmaes_syrk_plan(cfg: int, n: int, K: int):
    """(tiles, kspan, splits) of the mixed-precision split-k SYRK with tile
    configuration cfg (host only)."""
    t, ks, sp = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.cmaes_syrk_plan(int(cfg), int(n), int(K), C.byref(t), C.byref(ks), C.byref(sp)))
    return t.value, ks.value, sp.value


def _tune_key(n, lam, precision):
    return f"{cmaes_device_arch()}|n={n}|lam={lam}|precision={precision}"


class CMAES:
    """Owning wrapper of one handle (one descent plus its IPOP restarts)."""

    def __init__(self, n, lam=0, sigma0=2.0, seed=0, precision="mixed", objective=None, R=None,
                 xstar=None, allocator=None, **options):
        """allocator: None (hipMalloc) or "torch" (PyTorch's caching allocator,
        through the options' allocator hook)."""
        self.h = None
        self.allocator = None
        self.h = cmaes_create(n, lam, sigma0, seed)
        self.n = n
        opt = cmaes_default_options()
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        for k, v in options.items():
            if k == "stream":
                v = C.c_void_p(v) if v else None
            if k == "variant" and isinstance(v, str):
                v = VARIANTS[v]
            setattr(opt, k, v)
        if allocator == "torch":
            import torch
            stream = None
            if options.get("stream"):
                stream = torch.cuda.ExternalStream(int(options["stream"]))
            self.allocator = TorchAllocator(stream=stream)
            self.allocator.install(opt)
        elif allocator is not None:
            raise ValueError("allocator must be None or 'torch'")
        cmaes_set_options(self.h, opt)
        if objective is not None:
            cmaes_set_objective(self.h, objective, n, R, xstar)

    def close(self):
        if self.h:
            cmaes_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def lam(self):
        return self.state(arrays=False)["lambda"]

    def generation(self):
        cmaes_generation(self.h)

    def generation_with_z(self, Z):
        cmaes_generation_with_z(self.h, Z)

    def ask(self):
        s = self.state(arrays=False)
        return cmaes_ask(self.h, s["n"], s["lambda"])

    def tell(self, f):
        cmaes_tell(self.h, f)

    def restart_ipop(self):
        return cmaes_restart_ipop(self.h)

    def ipop_run(self):
        return cmaes_ipop_run(self.h)

    def state(self, arrays=True):
        return cmaes_state(self.h, arrays)

    def set_state(self, st):
        cmaes_set_state(self.h, st)

    def enable_timing(self, on=True):
        cmaes_enable_timing(self.h, on)

    def phase_times(self):
        return cmaes_phase_times(self.h)

    def enable_graphs(self, on=True):
        cmaes_enable_graphs(self.h, on)

    def set_eigen_correction(self, on=True, max_angle_norm=2e-3):
        cmaes_set_eigen_correction(self.h, on, max_angle_norm)

    def enable_kernel_timing(self, on=True):
        cmaes_enable_kernel_timing(self.h, on)

    def gemm_config(self, site):
        return cmaes_get_gemm_config(self.h, site)

    def set_gemm_config(self, site, cfg):
        cmaes_set_gemm_config(self.h, site, cfg)

    def autotune(self, reps=10, cache=None):
        """Select the float32 GEMM tiles for the current (n, lambda).

        With ``cache`` (a JSON file path) a previous choice for the same device
        architecture, shape and precision is reused and new choices are added.
        Returns {site: configuration}.
        """
        opt = cmaes_get_options(self.h)
        key = _tune_key(self.n, self.lam, int(opt.precision))
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        if key in table:
            for site, cfg in table[key]["chosen"].items():
                cmaes_set_gemm_config(self.h, site, cfg)
            return dict(table[key]["chosen"])
        us, chosen = cmaes_autotune(self.h, reps)
        res = dict(zip(SITES, chosen))
        if cache:
            table[key] = {"chosen": res, "us": us.tolist()}
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        self.last_tune_us = us
        return res

    def kernel_times(self):
        return cmaes_kernel_times(self.h)


def cmaes_batch_create(n, lam, sigma0, seed):
    k = len(n)
    arr_i = lambda v: (C.c_int * k)(*[int(x) for x in v])
    b = _lib.cmaes_batch_create(k, arr_i(n), arr_i(lam), (C.c_double * k)(*[float(x) for x in sigma0]),
                                (C.c_uint64 * k)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in seed]))
    if not b:
        raise CmaesError(CMAES_EINVAL, cmaes_last_error())
    return b


def cmaes_batch_destroy(b):
    _lib.cmaes_batch_destroy(b)


def cmaes_batch_count(b) -> int:
    return _check(_lib.cmaes_batch_count(b), allow=tuple(range(1, 1 << 20)))


def cmaes_batch_set_options(b, opt: CmaesOptions):
    _check(_lib.cmaes_batch_set_options(b, C.byref(opt)))


def cmaes_batch_set_objective(b, k, kind, n, R=None, xstar=None):
    kk = OBJECTIVES[kind] if isinstance(kind, str) else int(kind)
    Rf = _colmajor(R, (n, n)) if R is not None else None
    xs = np.ascontiguousarray(xstar, dtype=np.float64) if xstar is not None else None
    _check(_lib.cmaes_batch_set_objective(b, int(k), kk, _dptr(Rf), _dptr(xs)))


def cmaes_batch_generation(b):
    _check(_lib.cmaes_batch_generation(b))


def cmaes_batch_state(b, k, arrays: bool = True) -> dict:
    return cmaes_state(b, arrays, _fetch=lambda st: _lib.cmaes_batch_state(b, int(k), C.byref(st)))


def cmaes_batch_best(b):
    f = C.c_double(0.0)
    k = C.c_int(-1)
    _check(_lib.cmaes_batch_best(b, C.byref(f), C.byref(k)))
    return f.value, k.value


class CMAESBatch:
    """Owning wrapper of a batch of concurrent descents."""

    def __init__(self, n, lam, sigma0, seed, precision="mixed", **options):
        self.b = cmaes_batch_create(n, lam, sigma0, seed)
        self.n = list(n)
        opt = cmaes_default_options()
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        for k, v in options.items():
            if k == "variant" and isinstance(v, str):
                v = VARIANTS[v]
            setattr(opt, k, v)
        cmaes_batch_set_options(self.b, opt)

    def set_objective(self, k, kind, R=None, xstar=None):
        cmaes_batch_set_objective(self.b, k, kind, self.n[k], R, xstar)

    def enable_graphs(self, on=True):
        cmaes_batch_enable_graphs(self.b, on)

    def generation(self):
        cmaes_batch_generation(self.b)

    def state(self, k, arrays=True):
        return cmaes_batch_state(self.b, k, arrays)

    def best(self):
        return cmaes_batch_best(self.b)

    def close(self):
        if self.b:
            cmaes_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---- K-Replicated (Alg. 3) -------------------------------------------------

def cmaes_krep_create(n, lambda_start, k_max, sigma0, seed):
    r = _lib.cmaes_krep_create(int(n), int(lambda_start), int(k_max), float(sigma0), int(seed))
    if not r:
        raise CmaesError(CMAES_EINVAL, cmaes_last_error())
    return r


def cmaes_krep_destroy(r):
    _lib.cmaes_krep_destroy(r)


def cmaes_krep_set_options(r, opt: CmaesOptions):
    _check(_lib.cmaes_krep_set_options(r, C.byref(opt)))


def cmaes_krep_set_objective(r, kind, n, R=None, xstar=None):
    k = OBJECTIVES[kind] if isinstance(kind, str) else int(kind)
    Rm = _colmajor(R, (n, n)) if R is not None else None
    xs = np.ascontiguousarray(xstar, dtype=np.float64) if xstar is not None else None
    _check(_lib.cmaes_krep_set_objective(r, k, _dptr(Rm), _dptr(xs)))


def cmaes_krep_generation(r):
    _check(_lib.cmaes_krep_generation(r))


def cmaes_krep_run(r, max_lockstep_generations):
    _check(_lib.cmaes_krep_run(r, int(max_lockstep_generations)))


def cmaes_krep_status(r) -> dict:
    s = KrepStatus()
    _check(_lib.cmaes_krep_status(r, C.byref(s)))
    return {k: getattr(s, k) for k, _ in KrepStatus._fields_}


class KReplicated:
    """Owning wrapper of a K-Replicated run (binary tree of descents)."""

    def __init__(self, n, lambda_start=0, k_max=4, sigma0=2.0, seed=0, precision="mixed", objective=None,
                 R=None, xstar=None, **options):
        self.n = n
        self.r = cmaes_krep_create(n, lambda_start, k_max, sigma0, seed)
        opt = cmaes_default_options()
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        for k, v in options.items():
            setattr(opt, k, v)
        cmaes_krep_set_options(self.r, opt)
        if objective is not None:
            cmaes_krep_set_objective(self.r, objective, n, R, xstar)

    def generation(self):
        cmaes_krep_generation(self.r)

    def run(self, max_lockstep_generations):
        cmaes_krep_run(self.r, max_lockstep_generations)

    def status(self):
        return cmaes_krep_status(self.r)

    def close(self):
        if self.r:
            cmaes_krep_destroy(self.r)
            self.r = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
