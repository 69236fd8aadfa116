/*
 * cmaes_mi355x.h - C ABI of the MI355X (gfx950) IPOP-CMA-ES generation path.
 *
 * The library minimises a blackbox f: R^n -> R by probing points and reading
 * their values (paper Sec. 1, problem statement).  One call of
 * cmaes_generation() runs one CMA-ES iteration (Alg. 1 loop body, Sec. 2.1):
 * sample lambda points with eq. (1), evaluate them, rank them, update the
 * mean, the two evolution paths, the step size sigma and the covariance C with
 * the rank-one plus rank-mu update of eq. (2)/(3), and, every kappa
 * generations, re-run the eigendecomposition C = B D^2 B^T.  The restart loop
 * of Alg. 2 (Sec. 2.2) is cmaes_restart_ipop() / cmaes_ipop_run().
 *
 * Conventions
 *  - Every function returns CMAES_OK (0) or a negative CMAES_E* code; no
 *    exception crosses the ABI.  cmaes_last_error() returns a thread-local
 *    message describing the last failure.
 *  - Matrices are column-major.  Candidate k of a population is column k.
 *  - Unless stated otherwise every pointer argument is HOST memory owned by
 *    the caller; the library has finished reading or writing it when the
 *    call returns (every such copy completes before the return) and never
 *    keeps it.  All device memory is owned by the handle and freed by
 *    cmaes_destroy() / cmaes_batch_destroy(); it comes from hipMalloc, or
 *    from the caller's allocator hook (options.dev_malloc / dev_free).
 *  - Work is queued on the handle's HIP stream (options.stream, NULL = the
 *    library's own stream).  Calls that hand data back to the host
 *    synchronise that stream; cmaes_generation() itself may return before the
 *    device has finished.
 *  - A handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef CMAES_MI355X_H
#define CMAES_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define CMAES_OK 0
#define CMAES_EINVAL (-1)   /* bad argument (size, pointer, enum)            */
#define CMAES_ENOMEM (-2)   /* device or host allocation failed              */
#define CMAES_EDEVICE (-3)  /* HIP runtime error or no gfx950 device          */
#define CMAES_ESTATE (-4)   /* call not valid in the handle's current state   */
#define CMAES_EKMAX (-5)    /* restart would exceed K_max (Alg. 2 loop end)   */
#define CMAES_ENUMERIC (-6) /* the eigendecomposition met non-finite values     */

/* ---- enums -------------------------------------------------------------- */
typedef enum {
  CMAES_FP64 = 0,        /* every step in float64                              */
  CMAES_MIXED = 1,       /* sampling, fitness, rank-mu SYRK in float32 MFMA;
                            eigensolve, paths, sigma, C in float64             */
  CMAES_MIXED_BF16X3 = 2 /* as MIXED, y = B D z as three bf16 split products   */
} cmaes_precision_t;

/* CMA-ES variants; the paper names the active and the large-scale ones as
 * future work (Sec. 5):
 *  STANDARD  - positive rank weights only (the default);
 *  ACTIVE    - the covariance update also takes the worse half of the ranks
 *              with negative weights (each scaled by n / ||C^{-1/2} y||^2);
 *              mean and paths as STANDARD;
 *  SEPARABLE - C kept diagonal (sep-CMA-ES, linear time and memory per
 *              sample): y = D z elementwise, c1 and cmu times (n + 2) / 3,
 *              no eigendecomposition (B = I, D = sqrt(diag C)). */
typedef enum {
  CMAES_VARIANT_STANDARD = 0,
  CMAES_VARIANT_ACTIVE = 1,
  CMAES_VARIANT_SEPARABLE = 2
} cmaes_variant_t;

typedef enum {
  CMAES_OBJ_NONE = 0,      /* no fused objective: host ask/tell only           */
  CMAES_OBJ_SPHERE = 1,    /* sum_i u_i^2                                      */
  CMAES_OBJ_ELLIPSOID = 2, /* sum_i 10^(6 (i-1)/(n-1)) u_i^2                   */
  CMAES_OBJ_RASTRIGIN = 3  /* 10 n + sum_i (u_i^2 - 10 cos(2 pi u_i))          */
} cmaes_objective_t;       /* u = R (x - x*), R = I and x* = 0 when not given  */

/* Stop bits (reading of the stopping conditions named in Sec. 2.2). */
#define CMAES_STOP_TOLHISTFUN (1u << 0)
#define CMAES_STOP_TOLFUN (1u << 1)
#define CMAES_STOP_TOLX (1u << 2)
#define CMAES_STOP_NOEFFECTAXIS (1u << 3)
#define CMAES_STOP_NOEFFECTCOORD (1u << 4)
#define CMAES_STOP_CONDITIONCOV (1u << 5)
#define CMAES_STOP_FTARGET (1u << 6)
#define CMAES_STOP_MAXGEN (1u << 7)
#define CMAES_STOP_MAXEVALS (1u << 8)
#define CMAES_STOP_NUMERIC (1u << 9)

/* ---- options ------------------------------------------------------------ */
typedef struct {
  int32_t precision;      /* cmaes_precision_t (default CMAES_MIXED)              */
  int32_t eigen_interval; /* kappa; 0 = max(1, ceil(1/(10 n (c1+cmu))))          */
  int32_t k_max;          /* Alg. 2 K_max (default 256)                          */
  int32_t max_gens;       /* per descent; 0 = no limit                           */
  int64_t max_evals;      /* whole run (Alg. 2 'budget'); 0 = no limit            */
  double box_lo, box_hi;  /* search box of the initial mean (default [-4, 4])     */
  double f_target;        /* stop when best f < f_target (default 1e-8)           */
  double tol_hist_fun;    /* default 1e-12                                        */
  double tol_fun;         /* default 1e-12                                        */
  double tol_x_factor;    /* TolX = tol_x_factor * sigma0 (default 1e-12)         */
  double max_condition;   /* ConditionCov threshold on cond(C) (default 1e14)     */
  void* stream;           /* hipStream_t to run on; NULL = library-owned stream   */
  /* Device allocator hook (both NULL = hipMalloc / hipFree, the default).
   * dev_malloc(bytes, alloc_ctx) returns device memory of the current device
   * (NULL on failure -> CMAES_ENOMEM); dev_free(ptr, alloc_ctx) releases it.
   * The library synchronises the handle's stream before each release.  The
   * hook in effect at the handle's first allocation (its first generation,
   * state or objective call) serves the handle for its whole life; passing a
   * different hook after that is CMAES_ESTATE, setting only one of the two
   * functions CMAES_EINVAL.  The Python binding uses this to allocate from
   * PyTorch's caching allocator. */
  void* (*dev_malloc)(size_t bytes, void* alloc_ctx);
  void (*dev_free)(void* ptr, void* alloc_ctx);
  void* alloc_ctx;
  /* cmaes_variant_t (default CMAES_VARIANT_STANDARD); changeable before the
   * first generation only (CMAES_ESTATE otherwise). */
  int32_t variant;
  int32_t reserved_;      /* zero */
} cmaes_options_t;

/* Fill *opt with the defaults listed above.  Returns CMAES_EINVAL if opt is NULL. */
int cmaes_default_options(cmaes_options_t* opt);

/* ---- state snapshot ----------------------------------------------------- */
/* Scalars are always filled by cmaes_state().  Each pointer is an optional
 * caller-owned host buffer (NULL = not copied): m, p_sigma, p_c, D, x_best
 * hold n doubles; C and B hold n*n doubles (column-major); f holds lambda
 * doubles (fitness of the last generation, candidate order) and order holds
 * lambda int32 (order[r] = candidate of rank r, ascending f, ties by index,
 * NaN last).  cmaes_set_state() reads n, lambda, gen, sigma and every
 * non-NULL buffer among m, C, B, D, p_sigma, p_c; other fields are ignored. */
typedef struct {
  int32_t n, lambda, mu, restart;
  int64_t gen;         /* generations in the current descent                   */
  int64_t evals;       /* evaluations in the current descent                   */
  int64_t total_evals; /* evaluations over all descents of this handle         */
  double sigma;
  double f_best;       /* best f over all descents of this handle              */
  uint32_t stop;       /* CMAES_STOP_* bits of the current descent             */
  int32_t kappa;       /* eigendecomposition interval in use                   */
  int32_t eig_sweeps;  /* Jacobi sweeps used by the last eigendecomposition    */
  int32_t eig_corrections; /* closing corrections it used after the sweeps    */
  double* m;
  double* C;
  double* B;
  double* D;
  double* p_sigma;
  double* p_c;
  double* x_best;
  double* f;
  int32_t* order;
} cmaes_state_t;

typedef struct cmaes cmaes_t; /* opaque; create -> destroy */

/* Create a descent for dimension n (>= 1) and population lambda (<= 0 selects
 * 4 + floor(3 ln n); otherwise >= 2), initial step size sigma0 > 0 and a
 * 64-bit seed.  The initial mean is uniform in [box_lo, box_hi]^n drawn from
 * the seed (Sec. 4.1); C = B = D = I, p_sigma = p_c = 0.  Device memory is
 * allocated on the current HIP device.  Options may be changed with
 * cmaes_set_options() before the first generation.  Returns NULL on failure
 * (reason in cmaes_last_error()). */
cmaes_t* cmaes_create(int n, int lambda, double sigma0, uint64_t seed);

/* Free every resource of h (NULL is a no-op). */
void cmaes_destroy(cmaes_t* h);

/* Replace the options.  Changing precision or stream is only allowed before
 * the first generation of a descent (CMAES_ESTATE otherwise); a new box
 * redraws the initial mean if no generation has run yet. */
int cmaes_set_options(cmaes_t* h, const cmaes_options_t* opt);

/* Read the options in use into *opt. */
int cmaes_get_options(const cmaes_t* h, cmaes_options_t* opt);

/* Select the fused objective.  R: n*n column-major rotation (NULL = identity);
 * xstar: n values (NULL = origin).  Both are copied to the device. */
int cmaes_set_objective(cmaes_t* h, int kind, const double* R, const double* xstar);

/* One full generation on the device with the fused objective (Alg. 1 body).
 * Returns CMAES_ESTATE, and queues nothing, if no objective is set or the
 * descent has stopped: a stop test of the previous generation fired (the
 * call first waits for that generation's stop tests to finish on the
 * device).  cmaes_restart_ipop() and cmaes_set_state() clear the stop.
 * Returns CMAES_ENUMERIC if this generation's eigendecomposition met
 * non-finite values in C; the generation's stop tests have then run and set
 * CMAES_STOP_CONDITIONCOV (and CMAES_STOP_NUMERIC where m, sigma, p_c,
 * diag C or D is non-finite), so the next call returns CMAES_ESTATE. */
int cmaes_generation(cmaes_t* h);

/* Parity hook: as cmaes_generation() but with the n*lambda normal matrix Z
 * (column-major, column k = z_k of eq. (1)) supplied by the caller; Z has
 * been copied to the device when the call returns.  Same return codes. */
int cmaes_generation_with_z(cmaes_t* h, const double* Z);

/* Host blackbox path, first half: sample the generation's points
 * x_k = m + sigma B D z_k into X (n*lambda, column-major).  CMAES_ESTATE on
 * a stopped descent (as cmaes_generation). */
int cmaes_ask(cmaes_t* h, double* X);

/* Allocation-free variant of cmaes_ask(), for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): identical points, but staged in the library's
 * static device array (8 MiB on each device, held until the process ends)
 * instead of a buffer the handle allocates on its first ask.  It calls no
 * hipMalloc, hipFree or other allocating routine.  Returns CMAES_EINVAL if
 * n * lambda exceeds 1048576 (the array's doubles), CMAES_ESTATE if the
 * handle's buffers do not exist yet (any earlier cmaes_state,
 * cmaes_set_objective or generation call creates them) or the descent has
 * stopped.  All calls on one device share the array: calls on one device
 * that overlap in time (from different host threads) race. */
int cmaes_ask_noalloc(cmaes_t* h, double* X);

/* Host blackbox path, second half: supply the lambda fitness values of the
 * points returned by the last cmaes_ask() (NaN counts as +inf) and run the
 * rest of the generation.  CMAES_ESTATE without a pending ask;
 * CMAES_ENUMERIC as cmaes_generation. */
int cmaes_tell(cmaes_t* h, const double* f);

/* Alg. 2 restart: lambda <- 2 lambda (K <- 2K), a fresh mean from the seed
 * stream, sigma = sigma0, C = B = D = I, zero paths; the best point over all
 * descents is kept.  CMAES_EKMAX if 2K would exceed K_max (nothing changes). */
int cmaes_restart_ipop(cmaes_t* h);

/* Run Alg. 2 on the fused objective: generations until a stop bit fires
 * (a CMAES_ENUMERIC generation counts as stopped), then restart with doubled
 * lambda, until K > K_max, f_best < f_target or the evaluation budget is
 * spent.  Writes the number of descents run into
 * *descents (may be NULL).  Returns CMAES_OK when the loop ended normally. */
int cmaes_ipop_run(cmaes_t* h, int* descents);

/* Copy the state out (synchronises the stream).  See cmaes_state_t. */
int cmaes_state(const cmaes_t* h, cmaes_state_t* out);

/* Overwrite the state (test and resume hook).  n and lambda must match the
 * handle.  Clears the stop bits and the f-history of the descent. */
int cmaes_set_state(cmaes_t* h, const cmaes_state_t* in);

/* ---- batched concurrent descents (K-Distributed, Sec. 3.2.3) ------------
 * count independent descents of possibly different n and lambda that step
 * together: instance k is created like cmaes_create(n[k], lambda[k],
 * sigma0[k], seed[k]) and runs on its own HIP stream.  One batch generation
 * advances every instance by one generation; an instance whose stop tests
 * fired is then restarted with the same lambda (fresh mean from its seed
 * stream, restart index + 1), so the batch keeps its population sizes
 * (restart-on-finish, Sec. 5).  Returns NULL on failure. */
typedef struct cmaes_batch cmaes_batch_t;
cmaes_batch_t* cmaes_batch_create(int count, const int* n, const int* lambda, const double* sigma0,
                                  const uint64_t* seed);
void cmaes_batch_destroy(cmaes_batch_t* b);
/* Number of instances (or a negative error code). */
int cmaes_batch_count(const cmaes_batch_t* b);
/* Apply the options to every instance (the stream field is ignored). */
int cmaes_batch_set_options(cmaes_batch_t* b, const cmaes_options_t* opt);
/* Fused objective of instance k (as cmaes_set_objective). */
int cmaes_batch_set_objective(cmaes_batch_t* b, int k, int kind, const double* R, const double* xstar);
/* One generation of every instance, then restart-on-finish. */
/* Graph replay for every instance of the batch (see cmaes_enable_graphs). */
int cmaes_batch_enable_graphs(cmaes_batch_t* b, int on);
int cmaes_batch_generation(cmaes_batch_t* b);
/* State of instance k (as cmaes_state). */
int cmaes_batch_state(const cmaes_batch_t* b, int k, cmaes_state_t* out);
/* Best f over all instances and all their descents, and its instance. */
int cmaes_batch_best(const cmaes_batch_t* b, double* f_best, int* k_best);

/* Device time of the phases of the last generation in microseconds, measured
 * with HIP events when timing is enabled (cmaes_enable_timing).  out holds
 * CMAES_NUM_PHASES doubles: sample, fitness, rank, update, covariance, eigen. */
#define CMAES_NUM_PHASES 6
int cmaes_enable_timing(cmaes_t* h, int on);
int cmaes_phase_times(const cmaes_t* h, double* out);

/* Per-kernel device time while enabled (enabling resets the totals): the
 * float32 tile launches, the bf16 x 3 product (without its operand split) and
 * the Jacobi rounds record their own dispatch start and end timestamps; the
 * other kernels below are bracketed by HIP events.
 * cmaes_kernel_times() writes CMAES_NUM_KERNELS totals in microseconds and
 * launch counts, indexed by the CMAES_KERNEL_* values. */
#define CMAES_KERNEL_NORMALS 0     /* Philox + Box-Muller sampler               */
#define CMAES_KERNEL_SAMPLE_GEMM 1 /* Y = B D Z                                 */
#define CMAES_KERNEL_FITNESS 2     /* R Y with the objective epilogue           */
#define CMAES_KERNEL_RANK 3        /* argsort of f                              */
#define CMAES_KERNEL_SYRK 4        /* rank-mu SYRK (mixed: split-k products;    */
                                   /* float64: products + covariance epilogue)  */
#define CMAES_KERNEL_EIG_GEMM 5    /* float64 products of the eigensolver       */
#define CMAES_KERNEL_JACOBI 6      /* block-Jacobi rounds of the eigensolve     */
#define CMAES_KERNEL_SYRK_EPI 7    /* mixed: split-k sum + covariance epilogue  */
#define CMAES_NUM_KERNELS 8
/* Graph replay of the generation (Sec. 3.1 pipeline as one captured unit).
 * cmaes_generation (and the batch generation) queue the fixed part of a
 * generation -- sampling, fitness, ranking, recombination, paths, the
 * covariance update and the eigensolve set-up -- as one hipGraph, captured on
 * first use and replayed while the handle's shapes, stream, objective,
 * options and GEMM tiles are unchanged (any change re-captures).  The
 * eigensolve's sweeps and corrections, whose number depends on the data, are
 * replayed from graphs of their own between the host's convergence checks.
 * Results are bit-identical with graphs on or off.  Default on; graphs are
 * not used while phase or kernel timing is enabled, with caller-supplied z,
 * or on the legacy null stream. */
int cmaes_enable_graphs(cmaes_t* h, int on);
/* Closing correction of the eigensolve (C = B D^2 B^T, Sec. 2.1).  Once the
 * block-Jacobi sweeps have brought off(A) below 1e-8 of ||A||_F, one
 * simultaneous rotation of every index pair by its 2 x 2 Jacobi angle
 * (five float64 products) takes the place of the last sweep.  A correction
 * whose angles are not small (||Theta||_F > max_angle_norm) leaves A
 * unchanged and the solve finishes with sweeps.  Either way the solve stops
 * at the same off(A) <= 1e-13 ||A||_F.  on: 0 or 1 (default 1);
 * max_angle_norm in [0, 2e-3] (default 2e-3, the bound below which the
 * rotation is orthogonal to rounding; 0 rejects every correction that would
 * rotate).  CMAES_EINVAL outside that range.  cmaes_state() reports the
 * sweeps and corrections (rejected ones included) of the last eigensolve. */
int cmaes_set_eigen_correction(cmaes_t* h, int on, double max_angle_norm);
int cmaes_enable_kernel_timing(cmaes_t* h, int on);
int cmaes_kernel_times(const cmaes_t* h, double* total_us, int64_t* calls);

/* ---- float32 GEMM tiles and their tuner (Sec. 3.1 GEMM reformulation) -----
 * In CMAES_MIXED and CMAES_MIXED_BF16X3 the float32 MFMA products -- the
 * sampling product (B D) Z of eq. (1), the rotated-objective product R Y whose
 * epilogue reduces f, and the split-k rank-mu product of eq. (3) -- each run
 * one of CMAES_NUM_GEMM_CONFIGS block tiles (BM x BN x BK).  The tile changes
 * speed only: the sampling product is bit-identical for every tile; the
 * fitness and covariance sums change by float32 rounding.  CMAES_FP64 and the
 * bf16x3 sampling product have one tile and are not tuned.
 *
 * cmaes_gemm_config_info: the tile of configuration cfg (no device needed).
 * cmaes_set_gemm_config / cmaes_get_gemm_config: the tile of call site `site`
 *   (CMAES_SITE_*); CMAES_EINVAL for a tile the site cannot run (the
 *   covariance site takes square tiles only).  Default: configuration 0.
 * cmaes_autotune: times every configuration `reps` times at each tunable site
 *   on the handle's current (n, lambda) and keeps the fastest.  us (NULL or
 *   CMAES_NUM_SITES * cmaes_gemm_config_count() doubles, site-major) receives
 *   the mean microseconds per launch, -1 where not timed; chosen (NULL or
 *   CMAES_NUM_SITES) the selected configurations.  Leaves the search state
 *   untouched (the covariance site, split-k products plus epilogue, updates
 *   a scratch matrix instead of C); refused between ask and tell
 *   (CMAES_ESTATE).  Blocks until done.
 * cmaes_device_arch: the current device's architecture name (e.g. "gfx950"),
 *   NUL-terminated into buf of len bytes; the key of a tuning cache. */
#define CMAES_SITE_SAMPLE 0
#define CMAES_SITE_FITNESS 1
#define CMAES_SITE_SYRK 2
#define CMAES_NUM_SITES 3
#define CMAES_NUM_GEMM_CONFIGS 7
int cmaes_gemm_config_count(void);
int cmaes_gemm_config_info(int cfg, int32_t* bm, int32_t* bn, int32_t* bk);
int cmaes_set_gemm_config(cmaes_t* h, int site, int cfg);
int cmaes_get_gemm_config(const cmaes_t* h, int site, int32_t* cfg);
int cmaes_autotune(cmaes_t* h, int reps, double* us, int32_t* chosen);
int cmaes_device_arch(char* buf, int len);
/* Split-k plan of the mixed-precision rank-mu SYRK (eq. (3)) with tile
 * configuration cfg (a square one) on n x n with K = mu selected columns, host
 * only: the lower tiles, the k-range per split (a multiple of 32) and the
 * split count.  The products write splits * tiles * bm * bm float32 partial
 * sums that the covariance epilogue reads back.  CMAES_EINVAL for a
 * non-square cfg or n, K < 1. */
int cmaes_syrk_plan(int cfg, int n, int K, int32_t* tiles, int32_t* kspan, int32_t* splits);

/* ---- K-Replicated strategy (Sec. 3.2.2, Alg. 3) on one GPU ---------------
 * A binary tree of descents over one GPU's evaluation slots: k_max leaf
 * descents (lambda_start each, own seeds) start together; when both children
 * of a node have finished (any stop test), the node's descent starts with
 * twice their population size (an IPOP restart of the left child's handle;
 * the right child's handle is released), until the root descent
 * (lambda_start * k_max) finishes.  Every generation steps all running
 * descents in lockstep (fronts queued on per-descent streams, eigensolve
 * sweeps advanced together).  The run is done when the root finishes or the
 * best f found falls below f_target.
 *
 * cmaes_krep_create: k_max a power of two in [1, 1024]; lambda_start <= 0
 *   picks the default population size for n; NULL on failure.
 * cmaes_krep_set_options: applied to every descent (their streams are their
 *   own; k_max raised to the tree's); cmaes_krep_set_objective likewise.
 * cmaes_krep_generation: one lockstep generation, then the merges; a no-op
 *   once done.  cmaes_krep_run: generations until done or the limit.
 * cmaes_krep_status: running / finished descents, largest running lambda,
 *   lockstep generations, evaluations over all descents, best f, done. */
typedef struct cmaes_krep cmaes_krep_t;
typedef struct {
  int32_t running, finished, lambda_max_running, done;
  int64_t lockstep_generations, total_evals;
  double f_best;
} cmaes_krep_status_t;
cmaes_krep_t* cmaes_krep_create(int n, int lambda_start, int k_max, double sigma0, uint64_t seed);
void cmaes_krep_destroy(cmaes_krep_t* r);
int cmaes_krep_set_options(cmaes_krep_t* r, const cmaes_options_t* opt);
int cmaes_krep_set_objective(cmaes_krep_t* r, int kind, const double* R, const double* xstar);
int cmaes_krep_generation(cmaes_krep_t* r);
int cmaes_krep_run(cmaes_krep_t* r, int64_t max_lockstep_generations);
int cmaes_krep_status(const cmaes_krep_t* r, cmaes_krep_status_t* out);

/* Thread-local message for the last failing call (never NULL). */
const char* cmaes_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CMAES_MI355X_H */
