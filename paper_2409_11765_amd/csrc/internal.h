// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace cmx {

// Device-resident scalars of one descent.  Kernels read sigma and the
// generation counter from here, so a generation can be queued without any
// host round trip.
struct DevScalars {
  double sigma;       // step size (eq. (1))
  double f_best;      // best f over all descents of the handle
  double ps_norm;     // ||p_sigma|| after the update
  double hsig;        // 1 or 0 (p_c stall)
  double c_coef;      // a = 1 - c1 - cmu + (1-hsig) c1 cc (2-cc)
  double f_gen_min;   // fitness range of the current generation
  double f_gen_max;
  double sigma0;
  int64_t gen;        // generation within the descent
  int64_t evals;      // evaluations within the descent
  uint32_t stop;      // stop bits of the descent
  int32_t eig_ok;     // last eigendecomposition positive definite
  int32_t hist_count; // entries written into the f-history ring
  int32_t jac_sweeps; // sweeps used by the last eigensolve
  int32_t jac_corr;   // closing corrections among them
  int32_t pad_;
};

// Strategy parameters passed by value to kernels.
struct KParams {
  int n, lam, mu, kappa;
  double mueff, cs, ds, cc, c1, cmu, chin;
  double sumw;  // sum of the weights of all ranks (1, or less with active negative weights)
  int variant;  // cmaes_variant_t
};

struct StopParams {
  double tol_hist_fun, tol_fun, tolx, max_condition, f_target;
  int64_t max_gens, max_evals;
  int hist_len;
};

// ---- per-kernel event timer ------------------------------------------------
// When enabled, begin/end events are recorded around selected launches; the
// host folds them into per-kernel totals after the generation.
enum KernelId { KID_NORMALS = 0, KID_SAMPLE_GEMM, KID_FITNESS, KID_RANK, KID_SYRK, KID_EIG_GEMM,
                KID_JACOBI, KID_SYRK_EPI, KID_COUNT };
struct KTimer {
  static constexpr int kMax = 4096;
  bool on = false;
  int used = 0;
  hipStream_t st = nullptr;
  hipEvent_t ev[2 * kMax] = {};
  int kid[kMax] = {};
  double total_us[KID_COUNT] = {};
  int64_t calls[KID_COUNT] = {};
};
inline void kt_begin(KTimer* t, int kid) {
  if (!t || !t->on || t->used >= KTimer::kMax) return;
  t->kid[t->used] = kid;
  (void)hipEventRecord(t->ev[2 * t->used], t->st);
}
inline void kt_end(KTimer* t) {
  if (!t || !t->on || t->used >= KTimer::kMax) return;
  (void)hipEventRecord(t->ev[2 * t->used + 1], t->st);
  ++t->used;
}

// Event pair for a launch that records its own start and end timestamps
// (hipExtLaunchKernelGGL), so the measured duration is the kernel's alone,
// without the marker packets of kt_begin / kt_end.  False when not timing.
inline bool kt_ext(KTimer* t, int kid, hipEvent_t* start, hipEvent_t* stop) {
  if (!t || !t->on || t->used >= KTimer::kMax) return false;
  t->kid[t->used] = kid;
  *start = t->ev[2 * t->used];
  *stop = t->ev[2 * t->used + 1];
  ++t->used;
  return true;
}

// A launch that, while the kernel timer is on, records the dispatch's own
// start and end timestamps (hipExtLaunchKernelGGL), so its measured duration
// is the kernel's alone, without the marker packets of separate events.
template <typename... Formals, typename... Actuals>
void timed_launch(KTimer* kt, int kid, void (*kern)(Formals...), int grid, int block, hipStream_t st,
                  Actuals... args) {
  hipEvent_t t0, t1;
  if (kt_ext(kt, kid, &t0, &t1))
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, t0, t1, 0, static_cast<Formals>(args)...);
  else
    kern<<<grid, block, 0, st>>>(static_cast<Formals>(args)...);
}

// ---- error plumbing -------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
#define CMX_HIP(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      return ::cmx::fail(-3, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int round_up(int a, int b) { return ceil_div(a, b) * b; }

// ---- launchers (each queues work on `st` and returns a hipError_t) --------
// random numbers
hipError_t launch_normals(hipStream_t st, void* Z, bool fp64, int ldz, int n, int lam,
                          uint64_t seed, uint32_t restart, const DevScalars* sc);
hipError_t launch_init_mean(hipStream_t st, double* m, int n, double lo, double hi,
                            uint64_t seed, uint32_t restart);

// FP64 path: sampling GEMM Y = BD * Z, fitness GEMM on R*Y writing per-row-tile
// partial sums of the objective terms; without R (either precision) the
// objective is reduced from Y directly.
struct FitnessArgs {
  int kind;                 // cmaes_objective_t
  const double* d;          // n: R (m - x*) (or m - x*)
  const void* coef;         // n: per-row weights (ellipsoid), element type = T
  const DevScalars* sc;     // sigma
  void* partial;            // [row_tiles][lam] partial sums, element type = T
  int ld_partial;
};
hipError_t launch_sample_gemm_f64(hipStream_t st, int n, int lam, const double* BD, int ldbd, const double* Z,
                                  int ldz, double* Y, int ldy);
// y = (B D) z as bf16 x 3 split products with float32 accumulation; `work`
// holds the split operands (bf16x3_work_bytes(n, lam) bytes)
size_t bf16x3_work_bytes(int n, int lam);
hipError_t launch_sample_gemm_bf16x3(hipStream_t st, int n, int lam, const float* BD, int ldbd, const float* Z,
                                     int ldz, float* Y, int ldy, void* work, KTimer* kt, int kid);
hipError_t launch_fitness_gemm_f64(hipStream_t st, int n, int lam, const double* R, int ldr, const double* Y, int ldy,
                                   const FitnessArgs& fa, int* row_tiles);
hipError_t launch_fitness_direct(hipStream_t st, bool fp64, int n, int lam, const void* Y, int ldy,
                                 const FitnessArgs& fa, int* row_tiles);
hipError_t launch_fitness_reduce(hipStream_t st, bool fp64, int kind, int n, int lam,
                                 const void* partial, int ld_partial, int row_tiles, double* f);

// ranking
// order[r] = index of rank r (ascending f, ties by index, NaN last); work
// holds rank_work_elems(lam) int32: the sorted chunks and partial counts
hipError_t launch_rank(hipStream_t st, const double* f, int lam, int32_t* order, int32_t* work);
size_t rank_work_elems(int lam);

// recombination and vector updates
hipError_t launch_recombine(hipStream_t st, bool fp64, int n, int lam, int mu, const void* Y,
                            const void* Z, int ld, const int32_t* order, const double* w,
                            const double* sqrtw, void* Ysel, int ldsel, double* part_yw,
                            double* part_zw, int* nchunks);
hipError_t launch_reduce_yz(hipStream_t st, int n, int nchunks, const double* part_yw,
                            const double* part_zw, double* yw, double* zw);
hipError_t launch_matvec(hipStream_t st, int n, const double* B, int ldb, const double* x,
                         double* part, int* nchunks);
hipError_t launch_vec_update(hipStream_t st, const KParams& kp, int nchunks, const double* part_bz,
                             const double* yw, double* m, double* ps, double* pc, DevScalars* sc);
hipError_t launch_best(hipStream_t st, bool fp64, int n, int lam, const double* f,
                       const int32_t* order, const void* Y, int ldy, const double* m,
                       double* x_best, double* hist, int hist_len, DevScalars* sc);

// FP64 path covariance update C <- a C + c1 pc pc^T + cmu Ysel Ysel^T (lower
// tiles + mirror); the mixed paths use g32_syrk
void syrk_plan_f64(int n, int K, int* ntl, int* splits, int* kspan, size_t* work_elems);
// Ysel2: null, or the second operand (Ysel with signed columns)
hipError_t launch_syrk_update_f64(hipStream_t st, int n, int mu, const double* Ysel, const double* Ysel2, int ldsel,
                                  double* C, int ldc, const double* pc, double c1, double cmu, const DevScalars* sc,
                                  double* work);

// ---- tunable float32 MFMA GEMMs (mixed precisions) -------------------------
enum G32Site { G32_SAMPLE = 0, G32_FITNESS = 1, G32_SYRK = 2, G32_NUM_SITES = 3 };
struct G32Config {
  int bm, bn, bk;  // block tile
};
constexpr int kG32NumConfigs = 7;
extern const G32Config kG32Configs[kG32NumConfigs];
struct G32FitArgs {
  int kind;               // cmaes_objective_t
  const double* d;        // n: R (m - x*)
  const float* coef;      // n: ellipsoid weights
  const DevScalars* sc;   // sigma
};
bool g32_config_valid(int cfg, int site);
int g32_row_tiles(int cfg, int M);
// site G32_SAMPLE: out = A*B (float, ld ldo); G32_FITNESS: out = per-row-tile
// partial objective sums of d + sigma A*B ([row_tiles][N] floats, ld ldo)
// kt / kid: while kt is timing, the launch records its own start and end
// timestamps under kid
hipError_t g32_gemm(hipStream_t st, int cfg, int site, int M, int N, int K, const float* A, int lda, const float* B,
                    int ldb, void* out, int ldo, const G32FitArgs* fa, KTimer* kt = nullptr, int kid = 0);
void syrk32_plan(int cfg, int n, int K, int* ntl, int* splits, int* kspan, size_t* work_elems);
int syrk32_threads(int cfg);
size_t syrk32_max_work(int n, int K);
// C <- a C + c1 pc pc^T + cmu Y Y^T; partial_only stops after the split-k
// products (the tuner times that part alone, C is left untouched); kt (or
// null) times the products and the epilogue as KID_SYRK and KID_SYRK_EPI
hipError_t g32_syrk(hipStream_t st, int cfg, int n, int K, const float* Y, const float* Y2, int ldy, float* work,
                    double* C, int ldc, const double* pc, double c1, double cmu, const DevScalars* sc,
                    bool partial_only, KTimer* kt);

// generic FP64 GEMM: C = op(A) * op(B), column-major
hipError_t launch_dgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, const double* A,
                        int lda, const double* B, int ldb, double* C, int ldc);
// C = op(A) op(B) as two half-k products in one launch (two tiles per CU at
// n ~ 1000), the second into the n x n scratch W, then C += W; a plain
// launch_dgemm when the product has more tiles than the GPU has CUs
hipError_t launch_dgemm_ksplit(hipStream_t st, bool ta, bool tb, int M, int N, int K, const double* A, int lda,
                               const double* B, int ldb, double* C, int ldc, double* W, int ldw);
// C0 = A0 B and C1 = A1 B (no transposes) in one launch
hipError_t launch_dgemm2(hipStream_t st, int M, int N, int K, const double* A0, int lda0, const double* A1,
                         int lda1, const double* B, int ldb, double* C0, int ldc0, double* C1, int ldc1);

// eigensolver
struct EigWork {
  int N = 0;      // padded size (multiple of 32)
  int* gctl = nullptr;   // control block of a grouped solve (GC_WORDS ints, device memory)
  double* A = nullptr;   // N*N, ping-pong with A2
  double* A2 = nullptr;  // N*N
  double* V = nullptr;   // N*N
  double* Q = nullptr;   // (N/32) * 32*32, ping-pong with Q2
  double* Q2 = nullptr;
  double* T = nullptr;   // n*n scratch
  double* X1 = nullptr;  // N*N: angles, then the correction's rotation
  double* X2 = nullptr;  // N*N: products of the correction
  double* evals = nullptr;  // N
  int32_t* perm = nullptr;  // N
  double* sign = nullptr;   // N
  double* part = nullptr;   // 3 * max(n, tiles) partial sums
  double* scale = nullptr;  // max |a_ii|
  int* status = nullptr;  // [0] 1 converged, 2 sweep limit, 3 non-finite; [1] sweeps; [2] corrections
  int* hflags = nullptr;  // pinned host memory: [0] more sweeps needed, [1] non-finite,
                  // [2] off(A) small enough for a closing correction, [3] the last
                  // correction was rejected (its rotation was not small)
  int* dflags = nullptr;  // device address of hflags (written by the convergence test)
  // progress of the eigensolve in flight
  double *Acur = nullptr, *Anext = nullptr, *Qcur = nullptr, *Qnext = nullptr;
  int sweeps = 0;   // sweeps and corrections queued so far
  int corrections = 0;  // closing corrections among them
  int last_sweeps = 0;  // sweeps (not corrections) of the previous solve (0: none, or B replaced)
  bool last_closed = false;  // the previous solve ended with a correction
  bool fresh = true;  // the next sweep starts from A alone (no pair solves carried over)
  bool corr_queued = false;  // the last step queued was a correction
  bool corr_blocked = false;  // a correction was rejected: sweeps only for the rest of this solve
  bool correct_on = true;  // closing corrections enabled
  double corr_max_theta = 2e-3;  // acceptance bound on ||Theta||_F (graphs capture it)
  bool pending = false;
  // captured steps: [0] sweep from A, [1] from A2, [2] first sweep from A,
  // [3] from A2, [4] correction from A, [5] from A2
  hipGraphExec_t gx[6] = {};
  hipStream_t gstream = nullptr;
};
// Queue the warm start and the first convergence test; the host then
// synchronises the stream and calls eigen_step until it reports done (each
// call queues one more sweep, or the finishing kernels).
int eigen_begin(hipStream_t st, int n, const double* C, int ldc, const double* B, int ldb, EigWork& w, KTimer* kt);
// the host-side part of eigen_begin alone (after replaying its launches from a graph)
void eigen_begin_host(EigWork& w);
// ahead = true: queue the first batch of sweeps of a warm-started solve
// without reading the flags (no synchronisation needed; a no-op otherwise)
int eigen_step(hipStream_t st, int n, double* B, int ldb, double* D, void* BD, bool fp64_bd, int ldbd, EigWork& w,
               DevScalars* sc, int max_sweeps, KTimer* kt, bool use_graph, bool* done, bool ahead = false);
// release the captured sweep graphs (the stream or the buffers change)
void eigen_drop_graphs(EigWork& w);

// ---- grouped eigensolve: the sweeps of many descents in one launch per
// round, convergence decided per descent on the device (see eigen.hip)
constexpr int kGroupMax = 1024;  // descents per group
// padded size whose eigensolve, warm start included, runs whole in one
// workgroup (n <= 32): no separate warm-start launches are queued for it
constexpr int kWholeSolveN = 32;
constexpr int kGroupKinds = 5;   // launch kinds with per-descent workgroups
// words of a descent's control block (EigWork::gctl); k_offnorm_final of the
// warm start writes GC_MORE and GC_NONFIN
enum GroupCtl { GC_STOPR = 0, GC_MIN = 1, GC_LAST = 2, GC_MORE = 4, GC_NONFIN = 5, GC_DUE = 6, GC_WORDS = 8 };
struct GEigDesc {  // one descent of a grouped solve (device table entry)
  double *A, *A2, *V, *Q, *Q2, *part, *scale;
  const double* C;  // the covariance (read by the single-workgroup solve's warm start)
  int ldc;
  int* status;
  int* ctl;
  double* B;
  int ldb;
  double* D;
  void* BD;
  int ldbd;
  int bd64;  // B D stored in float64
  double* evals;
  int32_t* perm;
  double* sign;
  DevScalars* sc;
  int n, N;
};
struct GroupDueMask {  // bit i: descent i solves in this call
  uint32_t w[kGroupMax / 32];
};
__host__ __device__ inline bool due_mask_bit(const GroupDueMask& m, int i) { return (m.w[i >> 5] >> (i & 31)) & 1u; }
struct GroupEig {
  void* dtab = nullptr;   // device: GEigDesc[kGroupMax], then the workgroup offsets
  int* hflags = nullptr;  // pinned, mapped: [0] descents still sweeping, [1 + i] sweeps of descent i,
                          // [1 + kGroupMax + i] its status (1 converged, 2 sweep limit, 3 non-finite)
  int* dflags = nullptr;  // device address of hflags
  int* dactive = nullptr; // device memory: descents still sweeping (the last to stop zeroes hflags[0])
  int cap = 0, count = 0, pmax = 2;
  int nsmall = 0;         // descents with N = kWholeSolveN (solved whole by one workgroup each)
  int uq = 0, ur = 0;     // all descents of one size: pair-solve and tile / V workgroups each (else 0)
  std::vector<int> off;   // host copy of the offsets (kGroupKinds x (count + 1))
};
// (re)load the table of descents (their buffers must stay allocated while in use)
int group_eig_build(hipStream_t st, GroupEig& ge, const std::vector<GEigDesc>& descs);
// Solve the due descents, whose warm starts (eigen_begin) are already queued
// on `st` or ordered before it; ahead: sweeps to queue before the first wait.
// sweeps_out[i] receives the sweeps of due descent i, code_out[i] (may be
// null) its status: 1 converged, 2 sweep limit, 3 non-finite values.
int group_eig_solve(hipStream_t st, GroupEig& ge, const GroupDueMask& due, int max_sweeps, int ahead,
                    int* sweeps_out, int* code_out);
void group_eig_release(GroupEig& ge);

// workgroup w of a grouped launch belongs to entry i with off[i] <= w < off[i + 1]
// (the last entry with off[i] <= w).  First guess: the entry w would fall in
// if all entries were the same size, exact for a group of equal descents, so
// usually two dependent loads instead of a search of log2(count) of them.
__device__ __forceinline__ int group_find(const int* __restrict__ off, int count, int w) {
  int lo = 0, hi = count;
  if (count == 1) return 0;
  const int total = off[count];
  if (total > 0) {
    const int g = min(static_cast<int>(static_cast<int64_t>(w) * count / total), count - 1);
    const int a = off[g], b = off[g + 1];
    if (a <= w && w < b) return g;
    if (w < a)
      hi = g;
    else
      lo = g + 1;
  }
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= w)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// ---- grouped front: the fixed launches of a generation -- sampling to the
// eigensolve's warm start, and the stop tests -- for many descents of the
// mixed precision with a rotated fused objective, one launch per step for all
// of them (workgroups split over the descents by prefix sums, kind by kind)
enum GroupFrontKind {
  GF_NORMALS = 0, GF_SAMPLE, GF_SUB, GF_RMATVEC, GF_RVEC, GF_FITNESS, GF_FREDUCE, GF_RANK, GF_MERGE, GF_SCATTER,
  GF_BEST,
  GF_RECOMB, GF_REDYZ, GF_BMATVEC, GF_VECUPD, GF_SYRK, GF_SYRKEPI, GF_INIT, GF_OFFCOLS, GF_OFFFIN, GF_POLAR,
  GF_STOP, GF_KINDS
};
struct GFront {  // one descent (device table entry)
  int n, lam, mu, ldn, N;
  uint32_t k0, k1, restart;
  DevScalars* sc;
  uint32_t* hstop;  // device address of the host's mapped copy of the stop bits and f_best
  const float* BD;
  float* Z;
  float* Y;
  // d = R (m - x*)
  const double* Rd;
  double* m;
  const double* xstar;
  double* u;
  double* part_bz;
  double* d;
  // fitness
  int kind;
  int fit_tiles;
  const float* Rt;
  const float* coef;
  float* partial;
  double* f;
  // ranking, best point
  int32_t* rank_work;
  int32_t* order;
  double* x_best;
  double* hist;
  int hist_len;
  // recombination, paths, sigma
  const double* w;
  const double* sqrtw;
  float* Ysel;
  double* part_yw;
  double* part_zw;
  double* yw;
  double* zw;
  double* B;
  double* D;
  double* ps;
  double* pc;
  KParams kp;
  // covariance
  float* syrk_work;
  double* C;
  int syrk_ntl, syrk_splits, syrk_kspan;
  // eigensolve set-up and the re-orthogonalisation of B
  double *V, *A, *A2, *T, *epart, *scale;
  int* dflags;
  int* gctl;
  StopParams sp;
};
// one product C = op(A) op(B) per descent, n x n, as launch_dgemm_ksplit
// plans it (split: two half-k products into C and W, then C += W)
struct GDgemm {
  const double* A;
  int lda;
  const double* B;
  int ldb;
  double* C;
  int ldc;
  double* W;
  int ldw;
  int n, K0, split;
};
// launchers of the grouped steps; g / off: device table and this kind's
// offsets, wgs: this kind's total workgroups, mask: the descents that take
// part (the others' workgroups return at once)
hipError_t launch_group_normals(hipStream_t st, const GFront* g, const int* off, int count, int wgs);
hipError_t launch_group_g32(hipStream_t st, int cfg, int site, const GFront* g, const int* off, int count, int wgs);
hipError_t launch_group_syrk(hipStream_t st, int cfg, const GFront* g, const int* off_syrk, int wgs_syrk,
                             const int* off_epi, int wgs_epi, int count);
hipError_t launch_group_fitness_reduce(hipStream_t st, const GFront* g, const int* off, int count, int wgs);
hipError_t launch_group_update(hipStream_t st, int kind, const GFront* g, const int* off, int count, int wgs,
                               const GroupDueMask* mask);
hipError_t launch_group_dgemm(hipStream_t st, bool ta, const GDgemm* gd, const int* off_mm, int wgs_mm,
                              const int* off_add, int wgs_add, int count, const GroupDueMask& mask);
hipError_t launch_group_eigen_begin(hipStream_t st, int kind, const GFront* g, const int* off, int count, int wgs,
                                    const GroupDueMask& mask);
// syrk workgroups per descent (products, epilogue) for tile configuration cfg
void syrk32_group_wgs(int cfg, int n, int K, int* wgs_products, int* wgs_epi);
int g32_tiles(int cfg, int M, int N);
// workgroups of the rank's chunk sort and scatter, and of its merge counts
int rank_chunks(int lam);
int rank_merge_wgs(int lam);

// stop tests; the bits go to sc->stop and, when hstop is not null, to that
// word of pinned, mapped host memory (device address)
hipError_t launch_stop(hipStream_t st, const KParams& kp, const StopParams& sp, const double* m,
                       const double* C, int ldc, const double* B, int ldb, const double* D,
                       const double* pc, const double* hist, DevScalars* sc, uint32_t* hstop);

// variants (cmaes_variant_t)
// active: Ysel[:, r] = s_r y_{order[r]} and Ysig[:, r] = sign(w_r) Ysel[:, r]
// for the ranks r >= mu, s_r = sqrt(|w_r| n / ||z_{order[r]}||^2) (w_r = 0:
// zero columns), and Ysig[:, r] = Ysel[:, r] for r < mu
hipError_t launch_active_cols(hipStream_t st, bool fp64, int n, int lam, int mu, const void* Y, const void* Z, int ld,
                              const int32_t* order, const double* w_all, void* Ysel, void* Ysig, int ldsel);
// separable: Y = D z column by column (no product)
hipError_t launch_sep_sample(hipStream_t st, bool fp64, int n, int lam, const double* D, const void* Z, int ldz,
                             void* Y, int ldy);
// separable: C_ii <- c_coef C_ii + c1 pc_i^2 + cmu sum_{r<mu} w_r y_{i, order[r]}^2
hipError_t launch_sep_cov(hipStream_t st, bool fp64, int n, int mu, const void* Y, int ldy, const int32_t* order,
                          const double* w, const double* pc, double c1, double cmu, double* C, int ldc,
                          const DevScalars* sc);
// separable: D = sqrt(diag C), B D = diag(D) in the sampling precision, the
// decomposition's status (positive diagonal) into sc
hipError_t launch_sep_eigen(hipStream_t st, bool fp64, int n, const double* C, int ldc, double* D, void* BD, int ldbd,
                            DevScalars* sc);

// misc
// B <- (3 B - T) / 2 with T = B (B^T B) (Newton-Schulz step, rows < n)
hipError_t launch_polar_step(hipStream_t st, int n, double* B, int ldb, const double* T, int ldt);
hipError_t launch_set_identity(hipStream_t st, double* A, int n, int ld);
hipError_t launch_to_precision(hipStream_t st, bool fp64, const double* src, int ld_src, void* dst,
                               int ld_dst, int rows, int cols);
// d = R (m - x*) with R, x* optional; u and part are scratch (n and ceil(n/64) n)
hipError_t launch_shift(hipStream_t st, int n, const double* R, int ldr, const double* m, const double* xstar,
                        double* u, double* part, double* d);

}  // namespace cmx
