// C ABI: handle life cycle, the generation pipeline and the IPOP restart loop
// (Alg. 1 and Alg. 2 of the paper).  See include/cmaes_mi355x.h.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cmaes_mi355x.h"
#include "internal.h"

namespace cmx {

static thread_local std::string g_err = "no error";
void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace cmx

using namespace cmx;

static_assert(CMAES_NUM_GEMM_CONFIGS == kG32NumConfigs, "tile table and header disagree");
static_assert(CMAES_NUM_SITES == G32_NUM_SITES && CMAES_SITE_SYRK == G32_SYRK, "GEMM sites and header disagree");
static_assert(CMAES_NUM_KERNELS == KID_COUNT, "kernel ids and header disagree");

namespace {

// buffer epochs, unique over all handles of the process (a handle created at
// the address of a destroyed one never repeats its epoch)
std::atomic<uint64_t> g_epoch{1};

// tutorial default parameters (positive weights), identical to the oracle's reading
struct HostParams {
  KParams kp;
  std::vector<double> w, sqrtw;
  std::vector<double> w_all;  // all lam ranks: w, then 0 or the active negative weights
};

// variant (cmaes_variant_t): the active negative weights and the separable
// rates follow the same readings as the oracle's variants
HostParams make_params(int n, int lam, int kappa_opt, int variant = CMAES_VARIANT_STANDARD) {
  HostParams hp;
  KParams& k = hp.kp;
  k.n = n;
  k.lam = lam;
  k.mu = lam / 2;
  k.variant = variant;
  k.sumw = 1.0;
  hp.w.resize(k.mu);
  hp.sqrtw.resize(k.mu);
  double sw = 0.0;
  for (int i = 0; i < k.mu; ++i) {
    hp.w[i] = std::log((lam + 1) / 2.0) - std::log(static_cast<double>(i + 1));
    sw += hp.w[i];
  }
  double s2 = 0.0;
  for (int i = 0; i < k.mu; ++i) {
    hp.w[i] /= sw;
    s2 += hp.w[i] * hp.w[i];
    hp.sqrtw[i] = std::sqrt(hp.w[i]);
  }
  k.mueff = 1.0 / s2;
  k.cs = (k.mueff + 2.0) / (n + k.mueff + 5.0);
  k.ds = 1.0 + 2.0 * std::max(0.0, std::sqrt((k.mueff - 1.0) / (n + 1.0)) - 1.0) + k.cs;
  k.cc = (4.0 + k.mueff / n) / (n + 4.0 + 2.0 * k.mueff / n);
  k.c1 = 2.0 / ((n + 1.3) * (n + 1.3) + k.mueff);
  k.cmu = std::min(1.0 - k.c1, 2.0 * (k.mueff - 2.0 + 1.0 / k.mueff) / ((n + 2.0) * (n + 2.0) + k.mueff));
  k.chin = std::sqrt(static_cast<double>(n)) * (1.0 - 1.0 / (4.0 * n) + 1.0 / (21.0 * n * n));
  hp.w_all.assign(lam, 0.0);
  for (int i = 0; i < k.mu; ++i) hp.w_all[i] = hp.w[i];
  if (variant == CMAES_VARIANT_SEPARABLE) {
    k.c1 = std::min(1.0, k.c1 * (n + 2.0) / 3.0);
    k.cmu = std::min(1.0 - k.c1, k.cmu * (n + 2.0) / 3.0);
  }
  if (variant == CMAES_VARIANT_ACTIVE && k.cmu > 0.0) {
    // negative weights of the ranks beyond mu (an odd lam leaves rank mu+1 at 0)
    double sneg = 0.0, sneg2 = 0.0;
    std::vector<double> wn(lam - k.mu, 0.0);
    for (int i = k.mu; i < lam; ++i) {
      wn[i - k.mu] = std::min(0.0, std::log((lam + 1) / 2.0) - std::log(static_cast<double>(i + 1)));
      sneg += wn[i - k.mu];
      sneg2 += wn[i - k.mu] * wn[i - k.mu];
    }
    if (sneg < 0.0) {
      const double mueff_neg = sneg * sneg / sneg2;
      const double alpha = std::min({1.0 + k.c1 / k.cmu, 1.0 + 2.0 * mueff_neg / (k.mueff + 2.0),
                                     (1.0 - k.c1 - k.cmu) / (n * k.cmu)});
      double sum = 1.0;
      for (int i = k.mu; i < lam; ++i) {
        hp.w_all[i] = alpha * wn[i - k.mu] / -sneg;
        sum += hp.w_all[i];
      }
      k.sumw = sum;
    }
  }
  k.kappa = kappa_opt > 0 ? kappa_opt
                          : std::max(1, static_cast<int>(std::ceil(1.0 / (10.0 * n * (k.c1 + k.cmu)))));
  if (variant == CMAES_VARIANT_SEPARABLE) k.kappa = 1;
  return hp;
}

int default_lambda(int n) { return 4 + static_cast<int>(std::floor(3.0 * std::log(static_cast<double>(n)))); }

}  // namespace

struct cmaes {
  int n = 0, lam = 0, lam0 = 0, K = 1, restart = 0, ldn = 0;
  double sigma0 = 1.0;
  uint64_t seed = 0;
  cmaes_options_t opt{};
  hipStream_t st = nullptr;
  bool own_stream = false;
  int dev = 0;  // the HIP device the handle was created on
  // device allocator of every buffer of the handle, fixed at its first
  // allocation (options.dev_malloc / dev_free / alloc_ctx; null = hipMalloc)
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_ctx = nullptr;
  // stop bits of the last generation whose stop tests have run: the stop
  // kernel stores them into this pinned, mapped host word (hstop; dstop is
  // its device address), and ev_stop marks the end of that kernel
  uint32_t* hstop = nullptr;
  uint32_t* dstop = nullptr;
  hipEvent_t ev_stop = nullptr;
  bool stop_pending = false;  // ev_stop recorded and not yet waited for
  bool fp64 = false;
  HostParams hp;
  StopParams sp{};
  int64_t gen = 0, evals = 0, total_evals = 0;
  int obj_kind = CMAES_OBJ_NONE;
  bool have_R = false, have_xstar = false;
  std::vector<double> R_host, xstar_host;
  bool ask_pending = false;
  bool allocated = false;
  int cap_lam = 0, cap_mu = 0, hist_cap = 0;
  bool timing = false;
  hipEvent_t ev[CMAES_NUM_PHASES + 1] = {};
  double phase_us[CMAES_NUM_PHASES] = {};
  KTimer kt;
  bool eig_due = false;
  bool reorth_due = false;  // the eigen step starts by re-orthogonalising B
  int reorth_sweeps = 0;    // Jacobi sweeps applied to B since it was last orthogonal
  bool eig_uncounted = false;  // the last eigensolve's sweeps are not yet in reorth_sweeps
  int gcfg[G32_NUM_SITES] = {0, 0, 0};  // float32 GEMM tile per call site
  // captured front of a generation (sampling .. eigensolve set-up), one per
  // (eig_due, reorth_due) case, valid while gkey matches (see front_key)
  bool graphs = true;
  uint64_t epoch = 1;
  hipGraphExec_t gx[3] = {nullptr, nullptr, nullptr};
  uint64_t gkey[3] = {0, 0, 0};

  // float64 state
  DevScalars* sc = nullptr;
  double *m = nullptr, *ps = nullptr, *pc = nullptr, *C = nullptr, *B = nullptr, *D = nullptr;
  double *w = nullptr, *sqrtw = nullptr, *x_best = nullptr, *hist = nullptr, *d = nullptr;
  double *xstar = nullptr, *Rd = nullptr, *yw = nullptr, *zw = nullptr;
  double *part_yw = nullptr, *part_zw = nullptr, *part_bz = nullptr, *f = nullptr, *X = nullptr;
  int32_t* order = nullptr;
  int32_t* rank_work = nullptr;  // partial rank counts
  // sampling-precision buffers
  void *BD = nullptr, *Rt = nullptr, *Z = nullptr, *Y = nullptr, *Ysel = nullptr, *coef = nullptr;
  void* Ysig = nullptr;  // active: Ysel with the columns of negative weight negated
  void* partial = nullptr;
  void* syrk_work = nullptr;
  void* split = nullptr;  // bf16 hi / lo operands of the bf16 x 3 sampling product
  size_t split_cap = 0;
  double* u = nullptr;
  EigWork ew{};
  // small n: the eigensolve runs as a grouped solve of this one descent
  // (convergence tested on the device, several short sweeps per host wait)
  GroupEig ge1{};
  uint64_t ge1_epoch = 0;
};

namespace {

// Device buffer of the handle, zero-filled on the handle's stream (so the
// handle's kernels see the zeros without any other synchronisation).
template <typename P>
int dev_alloc(cmaes* h, P** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  void* q = nullptr;
  if (h->alloc_fn) {
    q = h->alloc_fn(bytes, h->alloc_ctx);
    if (!q) return fail(CMAES_ENOMEM, "caller allocator failed for " + std::to_string(bytes) + " bytes");
  } else if (hipMalloc(&q, bytes) != hipSuccess) {
    return fail(CMAES_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  *p = static_cast<P*>(q);
  CMX_HIP(hipMemsetAsync(q, 0, bytes, h->st));
  return 0;
}

// The caller must have synchronised the handle's stream (free_all and
// free_pop_buffers do): a caller allocator may hand the memory to other work
// at once.
template <typename P>
void dev_free(cmaes* h, P*& p) {
  if (p) {
    void* q = const_cast<void*>(static_cast<const void*>(p));
    if (h->free_fn)
      h->free_fn(q, h->alloc_ctx);
    else
      (void)hipFree(q);
  }
  p = nullptr;
}

size_t esz(const cmaes* h) { return h->fp64 ? sizeof(double) : sizeof(float); }

// f_best as of the handle's last stop tests: the mapped host copy the stop
// kernel writes next to the stop bits
double* host_fbest(const cmaes* h) { return reinterpret_cast<double*>(h->hstop + 2); }

void free_pop_buffers(cmaes* h) {
  if (h->st) (void)hipStreamSynchronize(h->st);  // nothing in flight uses the buffers
  dev_free(h, h->Z);
  dev_free(h, h->Y);
  dev_free(h, h->Ysel);
  dev_free(h, h->Ysig);
  dev_free(h, h->partial);
  dev_free(h, h->part_yw);
  dev_free(h, h->part_zw);
  dev_free(h, h->f);
  dev_free(h, h->X);
  dev_free(h, h->order);
  dev_free(h, h->rank_work);
  dev_free(h, h->w);
  dev_free(h, h->sqrtw);
  dev_free(h, h->hist);
  dev_free(h, h->syrk_work);
  dev_free(h, h->split);
  h->cap_lam = h->cap_mu = h->hist_cap = 0;
  h->split_cap = 0;
}

void drop_graphs(cmaes* h) {
  bool any = h->gx[0] || h->gx[1] || h->gx[2];
  for (auto g : h->ew.gx) any = any || g;
  if (any && h->st) (void)hipStreamSynchronize(h->st);  // no replay in flight
  eigen_drop_graphs(h->ew);
  for (int i = 0; i < 3; ++i) {
    if (h->gx[i]) (void)hipGraphExecDestroy(h->gx[i]);
    h->gx[i] = nullptr;
    h->gkey[i] = 0;
  }
  h->epoch = g_epoch.fetch_add(1);
}

void free_all(cmaes* h) {
  if (h->st) (void)hipStreamSynchronize(h->st);
  drop_graphs(h);
  free_pop_buffers(h);
  dev_free(h, h->sc);
  dev_free(h, h->m);
  dev_free(h, h->ps);
  dev_free(h, h->pc);
  dev_free(h, h->C);
  dev_free(h, h->B);
  dev_free(h, h->D);
  dev_free(h, h->x_best);
  dev_free(h, h->d);
  dev_free(h, h->u);
  dev_free(h, h->xstar);
  dev_free(h, h->Rd);
  dev_free(h, h->yw);
  dev_free(h, h->zw);
  dev_free(h, h->part_bz);
  dev_free(h, h->BD);
  dev_free(h, h->Rt);
  dev_free(h, h->coef);
  dev_free(h, h->ew.A);
  dev_free(h, h->ew.V);
  dev_free(h, h->ew.Q);
  dev_free(h, h->ew.T);
  dev_free(h, h->ew.A2);
  dev_free(h, h->ew.X1);
  dev_free(h, h->ew.X2);
  dev_free(h, h->ew.Q2);
  dev_free(h, h->ew.evals);
  dev_free(h, h->ew.perm);
  dev_free(h, h->ew.sign);
  dev_free(h, h->ew.part);
  dev_free(h, h->ew.scale);
  dev_free(h, h->ew.status);
  dev_free(h, h->ew.gctl);
  group_eig_release(h->ge1);
  h->ge1_epoch = 0;
  if (h->ew.hflags) (void)hipHostFree(h->ew.hflags);
  h->ew.hflags = nullptr;
  h->ew.dflags = nullptr;
  h->hstop = nullptr;
  h->dstop = nullptr;
  h->stop_pending = false;
  h->allocated = false;
}

int hist_len_for(int n, int lam) { return 10 + static_cast<int>(std::ceil(30.0 * n / lam)); }

void refresh_stop_params(cmaes* h) {
  StopParams& s = h->sp;
  s.tol_hist_fun = h->opt.tol_hist_fun;
  s.tol_fun = h->opt.tol_fun;
  s.tolx = h->opt.tol_x_factor * h->sigma0;
  s.max_condition = h->opt.max_condition;
  s.f_target = h->opt.f_target;
  s.max_gens = h->opt.max_gens;
  s.max_evals = 0;  // the evaluation budget is a whole-run limit checked by the host loop
  s.hist_len = hist_len_for(h->n, h->lam);
}

// split operands of the bf16 x 3 sampling product (that precision only; the
// precision may switch between the two float32 modes after allocation)
int alloc_split(cmaes* h) {
  const size_t need = h->opt.precision == CMAES_MIXED_BF16X3 ? bf16x3_work_bytes(h->n, h->lam) : 0;
  if (need <= h->split_cap) return 0;
  drop_graphs(h);
  if (h->st) (void)hipStreamSynchronize(h->st);  // nothing in flight uses the old buffer
  dev_free(h, h->split);
  h->split_cap = 0;
  if (int rc = dev_alloc(h, &h->split, need)) return rc;
  h->split_cap = need;
  return 0;
}

// population-size dependent buffers
int alloc_pop(cmaes* h) {
  const int n = h->n, ldn = h->ldn, lam = h->lam;
  // the rank-mu update runs over mu columns, or over all lam ranks (active)
  const bool active = h->opt.variant == CMAES_VARIANT_ACTIVE;
  const int mu = active ? lam : h->hp.kp.mu;
  if (lam <= h->cap_lam && mu <= h->cap_mu && hist_len_for(n, lam) <= h->hist_cap) return alloc_split(h);
  drop_graphs(h);
  free_pop_buffers(h);
  const size_t e = esz(h);
  int rc = 0;
  const int row_tiles = ceil_div(n, 64);
  if ((rc = dev_alloc(h, &h->Z, e * ldn * lam)) || (rc = dev_alloc(h, &h->Y, e * ldn * lam)) ||
      (rc = dev_alloc(h, &h->Ysel, e * ldn * mu)) || (rc = dev_alloc(h, &h->partial, 8ull * row_tiles * lam)) ||
      (rc = dev_alloc(h, &h->part_yw, 8ull * ceil_div(mu, 64) * n)) ||
      (rc = dev_alloc(h, &h->part_zw, 8ull * ceil_div(mu, 64) * n)) || (rc = dev_alloc(h, &h->f, 8ull * lam)) ||
      (rc = dev_alloc(h, &h->order, 4ull * lam)) || (rc = dev_alloc(h, &h->rank_work, 4ull * rank_work_elems(lam))) ||
      (rc = dev_alloc(h, &h->w, 8ull * lam)) || (rc = dev_alloc(h, &h->Ysig, active ? e * ldn * lam : 16)) ||
      (rc = dev_alloc(h, &h->sqrtw, 8ull * mu)) || (rc = dev_alloc(h, &h->hist, 8ull * hist_len_for(n, lam))))
    return rc;
  {
    int ntl, splits, kspan;
    size_t we;
    if (h->fp64)
      syrk_plan_f64(n, mu, &ntl, &splits, &kspan, &we);
    else
      we = syrk32_max_work(n, mu);
    if ((rc = dev_alloc(h, &h->syrk_work, e * we))) return rc;
  }
  h->cap_lam = lam;
  h->cap_mu = mu;
  h->hist_cap = hist_len_for(n, lam);
  return alloc_split(h);
}

int alloc_fixed(cmaes* h) {
  const int n = h->n, ldn = h->ldn;
  const size_t e = esz(h);
  const size_t nn = static_cast<size_t>(ldn) * n;
  const int N = round_up(n, 32);
  h->ew.N = N;
  int rc = 0;
  if ((rc = dev_alloc(h, &h->sc, sizeof(DevScalars))) || (rc = dev_alloc(h, &h->m, 8ull * ldn)) ||
      (rc = dev_alloc(h, &h->ps, 8ull * ldn)) || (rc = dev_alloc(h, &h->pc, 8ull * ldn)) ||
      (rc = dev_alloc(h, &h->C, 8 * nn)) || (rc = dev_alloc(h, &h->B, 8 * nn)) || (rc = dev_alloc(h, &h->D, 8ull * ldn)) ||
      (rc = dev_alloc(h, &h->x_best, 8ull * ldn)) || (rc = dev_alloc(h, &h->d, 8ull * ldn)) ||
      (rc = dev_alloc(h, &h->u, 8ull * ldn)) ||
      (rc = dev_alloc(h, &h->xstar, 8ull * ldn)) || (rc = dev_alloc(h, &h->Rd, 8 * nn)) ||
      (rc = dev_alloc(h, &h->yw, 8ull * ldn)) || (rc = dev_alloc(h, &h->zw, 8ull * ldn)) ||
      (rc = dev_alloc(h, &h->part_bz, 8ull * ceil_div(n, 64) * n)) || (rc = dev_alloc(h, &h->BD, e * nn)) ||
      (rc = dev_alloc(h, &h->Rt, e * nn)) || (rc = dev_alloc(h, &h->coef, e * ldn)) ||
      (rc = dev_alloc(h, &h->ew.A, 8ull * N * N)) || (rc = dev_alloc(h, &h->ew.V, 8ull * N * N)) ||
      (rc = dev_alloc(h, &h->ew.Q, 8ull * (N / 32) * 32 * 32)) || (rc = dev_alloc(h, &h->ew.T, 8 * nn)) ||
      (rc = dev_alloc(h, &h->ew.A2, 8ull * N * N)) || (rc = dev_alloc(h, &h->ew.Q2, 8ull * (N / 32) * 32 * 32)) ||
      (rc = dev_alloc(h, &h->ew.X1, 8ull * N * N)) || (rc = dev_alloc(h, &h->ew.X2, 8ull * N * N)) ||
      (rc = dev_alloc(h, &h->ew.evals, 8ull * N)) || (rc = dev_alloc(h, &h->ew.perm, 4ull * N)) ||
      (rc = dev_alloc(h, &h->ew.sign, 8ull * N)) || (rc = dev_alloc(h, &h->ew.scale, 16)) ||
      (rc = dev_alloc(h, &h->ew.status, 16)) || (rc = dev_alloc(h, &h->ew.gctl, 4ull * GC_WORDS)))
    return rc;
  {
    const int q = N / 32;
    if ((rc = dev_alloc(h, &h->ew.part, 8ull * 3 * std::max(n, q * (q + 1) / 2)))) return rc;
  }
  // convergence flags (words 0-3) and the stop bits (word 4): pinned, mapped
  // host memory the device writes directly
  void* hf = nullptr;
  if (hipHostMalloc(&hf, 32, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return fail(CMAES_ENOMEM, "hipHostMalloc failed");
  h->ew.hflags = static_cast<int*>(hf);
  for (int i = 0; i < 8; ++i) h->ew.hflags[i] = 0;
  void* dp = nullptr;
  if (hipHostGetDevicePointer(&dp, hf, 0) != hipSuccess) return fail(CMAES_EDEVICE, "hipHostGetDevicePointer failed");
  h->ew.dflags = static_cast<int*>(dp);
  h->hstop = reinterpret_cast<uint32_t*>(h->ew.hflags + 4);
  h->dstop = reinterpret_cast<uint32_t*>(h->ew.dflags + 4);
  return 0;
}

int upload_params(cmaes* h) {
  CMX_HIP(hipMemcpyAsync(h->w, h->hp.w_all.data(), 8 * h->hp.w_all.size(), hipMemcpyHostToDevice, h->st));
  CMX_HIP(hipMemcpyAsync(h->sqrtw, h->hp.sqrtw.data(), 8 * h->hp.sqrtw.size(), hipMemcpyHostToDevice, h->st));
  CMX_HIP(hipStreamSynchronize(h->st));
  return 0;
}

// objective-dependent device data in the sampling precision
int upload_objective_derived(cmaes* h);

int upload_objective(cmaes* h) {
  const int n = h->n;
  if (h->have_R)
    CMX_HIP(hipMemcpy2DAsync(h->Rd, 8ull * h->ldn, h->R_host.data(), 8ull * n, 8ull * n, n, hipMemcpyHostToDevice,
                             h->st));
  if (h->have_xstar)
    CMX_HIP(hipMemcpyAsync(h->xstar, h->xstar_host.data(), 8ull * n, hipMemcpyHostToDevice, h->st));
  return upload_objective_derived(h);  // synchronises the stream
}

int upload_objective_derived(cmaes* h) {
  const int n = h->n;
  std::vector<double> coef(n, 1.0);
  if (n > 1)
    for (int i = 0; i < n; ++i) coef[i] = std::pow(10.0, 6.0 * i / (n - 1));
  std::vector<float> cf(coef.begin(), coef.end());
  if (h->fp64)
    CMX_HIP(hipMemcpyAsync(h->coef, coef.data(), 8ull * n, hipMemcpyHostToDevice, h->st));
  else
    CMX_HIP(hipMemcpyAsync(h->coef, cf.data(), 4ull * n, hipMemcpyHostToDevice, h->st));
  if (h->have_R) CMX_HIP(launch_to_precision(h->st, h->fp64, h->Rd, h->ldn, h->Rt, h->ldn, n, n));
  CMX_HIP(hipStreamSynchronize(h->st));  // the host vectors are consumed before they go out of scope
  return 0;
}

// fresh descent: Alg. 2 initialisation line
int init_descent(cmaes* h, bool fresh) {
  const int n = h->n;
  DevScalars s{};
  CMX_HIP(hipMemcpyAsync(&s, h->sc, sizeof(s), hipMemcpyDeviceToHost, h->st));
  CMX_HIP(hipStreamSynchronize(h->st));
  const double f_best = fresh ? HUGE_VAL : s.f_best;
  std::memset(&s, 0, sizeof(s));
  s.sigma = h->sigma0;
  s.sigma0 = h->sigma0;
  s.f_best = f_best;
  s.eig_ok = 1;
  CMX_HIP(hipMemcpyAsync(h->sc, &s, sizeof(s), hipMemcpyHostToDevice, h->st));
  CMX_HIP(launch_init_mean(h->st, h->m, n, h->opt.box_lo, h->opt.box_hi, h->seed, static_cast<uint32_t>(h->restart)));
  CMX_HIP(hipMemsetAsync(h->ps, 0, 8ull * h->ldn, h->st));
  CMX_HIP(hipMemsetAsync(h->pc, 0, 8ull * h->ldn, h->st));
  CMX_HIP(launch_set_identity(h->st, h->C, n, h->ldn));
  CMX_HIP(launch_set_identity(h->st, h->B, n, h->ldn));
  std::vector<double> ones(n, 1.0);
  CMX_HIP(hipMemcpyAsync(h->D, ones.data(), 8ull * n, hipMemcpyHostToDevice, h->st));
  CMX_HIP(launch_to_precision(h->st, h->fp64, h->B, h->ldn, h->BD, h->ldn, n, n));
  CMX_HIP(hipMemsetAsync(h->ew.gctl, 0, 4ull * GC_WORDS, h->st));  // no previous solve
  CMX_HIP(hipStreamSynchronize(h->st));  // s and ones are consumed
  *h->hstop = 0;
  *host_fbest(h) = f_best;
  h->stop_pending = false;
  h->gen = 0;
  h->evals = 0;
  h->ask_pending = false;
  h->reorth_sweeps = 0;  // B = I
  h->eig_uncounted = false;
  h->ew.last_sweeps = 0;
  h->ew.last_closed = false;
  refresh_stop_params(h);
  return 0;
}

int ensure_ready(cmaes* h) {
  if (h->allocated) return alloc_pop(h);
  h->fp64 = (h->opt.precision == CMAES_FP64);
  h->alloc_fn = h->opt.dev_malloc;
  h->free_fn = h->opt.dev_free;
  h->alloc_ctx = h->opt.alloc_ctx;
  int rc;
  if ((rc = alloc_fixed(h)) || (rc = alloc_pop(h))) {
    free_all(h);
    return rc;
  }
  h->allocated = true;
  if ((rc = upload_params(h)) || (rc = init_descent(h, true))) return rc;
  if (h->obj_kind != CMAES_OBJ_NONE && (rc = upload_objective(h))) return rc;
  return 0;
}

void rec(cmaes* h, int i) {
  if (h->timing) (void)hipEventRecord(h->ev[i], h->st);
}

int phase_sample(cmaes* h, const double* Zhost) {
  const int n = h->n, lam = h->lam, ldn = h->ldn;
  rec(h, 0);
  if (Zhost) {
    // caller-supplied z: stage as float64 then convert to the sampling precision
    if (h->fp64) {
      CMX_HIP(hipMemcpy2DAsync(h->Z, 8ull * ldn, Zhost, 8ull * n, 8ull * n, lam, hipMemcpyHostToDevice, h->st));
      CMX_HIP(hipStreamSynchronize(h->st));  // the caller's buffer is consumed before the call returns
    } else {
      std::vector<float> zf(static_cast<size_t>(ldn) * lam, 0.0f);
      for (int k = 0; k < lam; ++k)
        for (int i = 0; i < n; ++i) zf[static_cast<size_t>(k) * ldn + i] = static_cast<float>(Zhost[static_cast<size_t>(k) * n + i]);
      CMX_HIP(hipMemcpyAsync(h->Z, zf.data(), 4ull * zf.size(), hipMemcpyHostToDevice, h->st));
      CMX_HIP(hipStreamSynchronize(h->st));
    }
  } else {
    kt_begin(&h->kt, KID_NORMALS);
    CMX_HIP(launch_normals(h->st, h->Z, h->fp64, ldn, n, lam, h->seed, static_cast<uint32_t>(h->restart), h->sc));
    kt_end(&h->kt);
  }
  // the float32 and bf16 x 3 products time themselves (their dispatches' own
  // timestamps; for bf16 x 3 the product alone, not the operand split)
  const bool self_timed = h->opt.variant != CMAES_VARIANT_SEPARABLE && !h->fp64;
  if (!self_timed) kt_begin(&h->kt, KID_SAMPLE_GEMM);
  if (h->opt.variant == CMAES_VARIANT_SEPARABLE)
    CMX_HIP(launch_sep_sample(h->st, h->fp64, n, lam, h->D, h->Z, ldn, h->Y, ldn));
  else if (h->opt.precision == CMAES_MIXED_BF16X3)
    CMX_HIP(launch_sample_gemm_bf16x3(h->st, n, lam, static_cast<const float*>(h->BD), ldn,
                                      static_cast<const float*>(h->Z), ldn, static_cast<float*>(h->Y), ldn,
                                      h->split, &h->kt, KID_SAMPLE_GEMM));
  else if (h->fp64)
    CMX_HIP(launch_sample_gemm_f64(h->st, n, lam, static_cast<const double*>(h->BD), ldn,
                                   static_cast<const double*>(h->Z), ldn, static_cast<double*>(h->Y), ldn));
  else
    CMX_HIP(g32_gemm(h->st, h->gcfg[G32_SAMPLE], G32_SAMPLE, n, lam, n, static_cast<const float*>(h->BD), ldn,
                     static_cast<const float*>(h->Z), ldn, h->Y, ldn, nullptr, &h->kt, KID_SAMPLE_GEMM));
  if (!self_timed) kt_end(&h->kt);
  rec(h, 1);
  return 0;
}

int phase_fitness(cmaes* h) {
  const int n = h->n, lam = h->lam, ldn = h->ldn;
  CMX_HIP(launch_shift(h->st, n, h->have_R ? h->Rd : nullptr, ldn, h->m, h->have_xstar ? h->xstar : nullptr, h->u,
                       h->part_bz, h->d));
  FitnessArgs fa{h->obj_kind, h->d, h->coef, h->sc, h->partial, lam};
  int tiles = 0;
  const bool g32 = h->have_R && !h->fp64;  // the float32 tile launch times itself
  if (!g32) kt_begin(&h->kt, KID_FITNESS);
  if (g32) {
    const G32FitArgs ga{h->obj_kind, h->d, static_cast<const float*>(h->coef), h->sc};
    tiles = g32_row_tiles(h->gcfg[G32_FITNESS], n);
    CMX_HIP(g32_gemm(h->st, h->gcfg[G32_FITNESS], G32_FITNESS, n, lam, n, static_cast<const float*>(h->Rt), ldn,
                     static_cast<const float*>(h->Y), ldn, h->partial, lam, &ga, &h->kt, KID_FITNESS));
  } else if (h->have_R)
    CMX_HIP(launch_fitness_gemm_f64(h->st, n, lam, static_cast<const double*>(h->Rt), ldn,
                                    static_cast<const double*>(h->Y), ldn, fa, &tiles));
  else
    CMX_HIP(launch_fitness_direct(h->st, h->fp64, n, lam, h->Y, ldn, fa, &tiles));
  if (!g32) kt_end(&h->kt);
  CMX_HIP(launch_fitness_reduce(h->st, h->fp64, h->obj_kind, n, lam, h->partial, lam, tiles, h->f));
  return 0;
}

// ranking, recombination, paths / sigma and the covariance update; the
// eigensolve (if due) is begun here and finished by eigen_drive or the
// batch driver
int phase_update_pre(cmaes* h) {
  const int n = h->n, lam = h->lam, ldn = h->ldn, mu = h->hp.kp.mu;
  rec(h, 2);
  kt_begin(&h->kt, KID_RANK);
  CMX_HIP(launch_rank(h->st, h->f, lam, h->order, h->rank_work));
  kt_end(&h->kt);
  CMX_HIP(launch_best(h->st, h->fp64, n, lam, h->f, h->order, h->Y, ldn, h->m, h->x_best, h->hist, h->sp.hist_len, h->sc));
  rec(h, 3);
  int nch = 0, nchb = 0;
  CMX_HIP(launch_recombine(h->st, h->fp64, n, lam, mu, h->Y, h->Z, ldn, h->order, h->w, h->sqrtw, h->Ysel, ldn,
                           h->part_yw, h->part_zw, &nch));
  CMX_HIP(launch_reduce_yz(h->st, n, nch, h->part_yw, h->part_zw, h->yw, h->zw));
  CMX_HIP(launch_matvec(h->st, n, h->B, ldn, h->zw, h->part_bz, &nchb));
  CMX_HIP(launch_vec_update(h->st, h->hp.kp, nchb, h->part_bz, h->yw, h->m, h->ps, h->pc, h->sc));
  rec(h, 4);
  const int variant = h->opt.variant;
  // the rank-mu operands: mu columns, or all lam ranks with signed copies (active)
  int K = mu;
  const void* Y2 = nullptr;
  if (variant == CMAES_VARIANT_ACTIVE) {
    CMX_HIP(launch_active_cols(h->st, h->fp64, n, lam, mu, h->Y, h->Z, ldn, h->order, h->w, h->Ysel, h->Ysig, ldn));
    K = lam;
    Y2 = h->Ysig;
  }
  if (variant == CMAES_VARIANT_SEPARABLE) {
    CMX_HIP(launch_sep_cov(h->st, h->fp64, n, mu, h->Y, ldn, h->order, h->w, h->pc, h->hp.kp.c1, h->hp.kp.cmu, h->C,
                           ldn, h->sc));
  } else if (h->fp64) {
    kt_begin(&h->kt, KID_SYRK);
    CMX_HIP(launch_syrk_update_f64(h->st, n, K, static_cast<const double*>(h->Ysel), static_cast<const double*>(Y2),
                                   ldn, h->C, ldn, h->pc, h->hp.kp.c1, h->hp.kp.cmu, h->sc,
                                   static_cast<double*>(h->syrk_work)));
    kt_end(&h->kt);
  } else {
    CMX_HIP(g32_syrk(h->st, h->gcfg[G32_SYRK], n, K, static_cast<const float*>(h->Ysel),
                     static_cast<const float*>(Y2), ldn, static_cast<float*>(h->syrk_work), h->C, ldn, h->pc,
                     h->hp.kp.c1, h->hp.kp.cmu, h->sc, false, &h->kt));
  }
  rec(h, 5);
  if (variant == CMAES_VARIANT_SEPARABLE)  // D = sqrt(diag C) after every update, B = I
    return launch_sep_eigen(h->st, h->fp64, n, h->C, ldn, h->D, h->BD, ldn, h->sc) == hipSuccess
               ? 0
               : fail(CMAES_EDEVICE, "separable decomposition launch failed");
  if (!h->eig_due) return 0;
  if (h->reorth_due) {
    // B drifts from orthogonality by the rounding of each eigensolve's
    // rotations (B = B_old V); one Newton-Schulz step B <- B (3 I - B^T B) / 2
    // removes the accumulated drift (to second order) before the warm start
    kt_begin(&h->kt, KID_EIG_GEMM);
    CMX_HIP(launch_dgemm_ksplit(h->st, true, false, n, n, n, h->B, ldn, h->B, ldn, h->ew.A2, h->ew.N, h->ew.X2,
                                h->ew.N));  // G = B^T B
    kt_end(&h->kt);
    kt_begin(&h->kt, KID_EIG_GEMM);
    CMX_HIP(launch_dgemm_ksplit(h->st, false, false, n, n, n, h->B, ldn, h->ew.A2, h->ew.N, h->ew.T, ldn, h->ew.X2,
                                h->ew.N));  // T = B G
    kt_end(&h->kt);
    CMX_HIP(launch_polar_step(h->st, n, h->B, ldn, h->ew.T, ldn));
  }
  if (h->ew.N == kWholeSolveN) {  // the single-workgroup solve forms its own warm start
    eigen_begin_host(h->ew);
    return 0;
  }
  return eigen_begin(h->st, n, h->C, ldn, h->B, ldn, h->ew, &h->kt);
}

// host-side counters of the generation just queued; eig_due and reorth_due
// must be set (set_due) before its launches are queued
bool due_next(const cmaes* h) { return (h->gen + 1) % h->hp.kp.kappa == 0; }
// B's drift from orthogonality grows with the rotation sweeps applied to it
// (B = B_old V per eigensolve): an eigen step re-orthogonalises B first once
// kReorthSweeps sweeps have accumulated since B was last orthogonal
constexpr int kReorthSweeps = 48;
void set_due(cmaes* h) {
  if (h->eig_uncounted) {  // the previous generation's eigensolve has finished
    h->reorth_sweeps += h->ew.sweeps;
    h->eig_uncounted = false;
  }
  h->eig_due = due_next(h) && h->opt.variant != CMAES_VARIANT_SEPARABLE;
  h->reorth_due = h->eig_due && h->reorth_sweeps >= kReorthSweeps;
  if (h->reorth_due) h->reorth_sweeps = 0;
  if (h->eig_due) h->eig_uncounted = true;
}
void advance_counters(cmaes* h) {
  h->gen += 1;
  h->evals += h->lam;
  h->total_evals += h->lam;
}

// one step of the eigensolve in flight (the stream must have been
// synchronised since the last call); *done once the decomposition is final
int eigen_advance(cmaes* h, bool* done, bool ahead = false) {
  // a decomposition that does not converge within the sweep limit (or meets
  // non-finite values) clears eig_ok on the device, which raises the
  // ConditionCov stop bit
  return eigen_step(h->st, h->n, h->B, h->ldn, h->D, h->BD, h->fp64, h->ldn, h->ew, h->sc, 40, &h->kt,
                    h->graphs && h->st != nullptr && !h->timing, done, ahead);
}
// the eigensolve of the generation just queued: its first batch of sweeps
// goes in behind the warm start, then one host check per step
int eigen_run(cmaes* h) {
  bool done = false;
  if (int rc = eigen_advance(h, &done, true)) return rc;
  while (!done) {
    CMX_HIP(hipStreamSynchronize(h->st));
    if (int rc = eigen_advance(h, &done)) return rc;
  }
  return 0;
}

// stop tests, then fold the optional timers
int phase_update_post(cmaes* h) {
  CMX_HIP(launch_stop(h->st, h->hp.kp, h->sp, h->m, h->C, h->ldn, h->B, h->ldn, h->D, h->pc, h->hist, h->sc,
                      h->dstop));
  CMX_HIP(hipEventRecord(h->ev_stop, h->st));
  h->stop_pending = true;
  rec(h, 6);
  if (h->kt.on && h->kt.used > 0) {
    CMX_HIP(hipEventSynchronize(h->kt.ev[2 * h->kt.used - 1]));
    for (int i = 0; i < h->kt.used; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, h->kt.ev[2 * i], h->kt.ev[2 * i + 1]);
      h->kt.total_us[h->kt.kid[i]] += 1000.0 * ms;
      h->kt.calls[h->kt.kid[i]] += 1;
    }
    h->kt.used = 0;
  }
  if (h->timing) {
    CMX_HIP(hipEventSynchronize(h->ev[6]));
    float ms = 0.f;
    // phases: sample | fitness | rank | update | covariance | eigen
    for (int i = 0; i < CMAES_NUM_PHASES; ++i) {
      (void)hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]);
      h->phase_us[i] = 1000.0 * ms;
    }
  }
  return 0;
}

// the generation's eigendecomposition met non-finite values: its stop tests
// have run (NUMERIC / CONDITIONCOV set); the call reports CMAES_ENUMERIC
int numeric_failure(const cmaes* h) {
  return fail(CMAES_ENUMERIC, "the eigendecomposition met non-finite values; the descent has stopped");
}

GEigDesc eig_desc(cmaes* h);

// dimensions whose eigensolve runs as a grouped solve of one descent: a sweep
// is one to three rounds there, so several are queued per host wait
constexpr int kSmallEigenN = 64;

// the eigensolve of the generation just queued, as a grouped solve of this
// descent (no closing correction); *nonfinite when it met non-finite values
int eigen_run_small(cmaes* h, bool* nonfinite) {
  if (h->ge1_epoch != h->epoch || h->ge1.count != 1) {
    if (int rc = group_eig_build(h->st, h->ge1, std::vector<GEigDesc>{eig_desc(h)})) return rc;
    h->ge1_epoch = h->epoch;
  }
  GroupDueMask due{};
  due.w[0] = 1u;
  const int last = h->ew.last_sweeps;
  int sweeps = 0, code = 1;
  if (int rc = group_eig_solve(h->st, h->ge1, due, 40, last >= 2 ? last - 1 : 0, &sweeps, &code)) return rc;
  h->ew.sweeps = sweeps;
  h->ew.corrections = 0;
  h->ew.last_sweeps = sweeps;
  h->ew.last_closed = false;
  h->ew.pending = false;
  *nonfinite = code == 3;
  return 0;
}

// the rest of a generation after its front: the eigensolve if due, then the
// stop tests
int finish_generation(cmaes* h) {
  bool nonfinite = false;
  if (h->eig_due) {
    if (h->ew.N <= kSmallEigenN) {
      if (int rc = eigen_run_small(h, &nonfinite)) return rc;
    } else {
      if (int rc = eigen_run(h)) return rc;
      nonfinite = h->ew.hflags[1] != 0;
    }
  }
  if (int rc = phase_update_post(h)) return rc;
  return nonfinite ? numeric_failure(h) : 0;
}

int phase_update(cmaes* h) {
  set_due(h);
  if (int rc = phase_update_pre(h)) return rc;
  advance_counters(h);
  return finish_generation(h);
}

// CMAES_ESTATE once a stop test of the descent has fired: waits for the stop
// tests of the last generation (the end of its queued work) and reads their
// bits from the mapped host word
int check_running(cmaes* h) {
  if (h->stop_pending) {
    CMX_HIP(hipEventSynchronize(h->ev_stop));
    h->stop_pending = false;
  }
  const uint32_t bits = __atomic_load_n(h->hstop, __ATOMIC_ACQUIRE);
  if (bits != 0)
    return fail(CMAES_ESTATE, "the descent has stopped (stop bits 0x" + [bits] {
      char b[16];
      std::snprintf(b, sizeof b, "%x", bits);
      return std::string(b);
    }() + "); restart it or reset its state");
  return 0;
}

int check(const cmaes* h) {
  if (!h) return fail(CMAES_EINVAL, "null handle");
  return 0;
}

// everything a captured front depends on besides device memory contents:
// buffer addresses (epoch), launch shapes and the host-side kernel arguments
uint64_t front_key(const cmaes* h, bool due) {
  uint64_t k = h->epoch;
  auto mix = [&k](uint64_t v) { k = (k ^ v) * 0x100000001B3ull + 0x9E3779B97F4A7C15ull; };
  mix(static_cast<uint64_t>(h->lam));
  mix(static_cast<uint64_t>(h->restart));
  mix(reinterpret_cast<uintptr_t>(h->st));
  mix(static_cast<uint64_t>(h->obj_kind) | (h->have_R ? 16u : 0u) | (h->have_xstar ? 32u : 0u));
  mix(static_cast<uint64_t>(h->opt.precision));
  mix(static_cast<uint64_t>(h->opt.variant) + 7);
  for (int i = 0; i < G32_NUM_SITES; ++i) mix(static_cast<uint64_t>(h->gcfg[i]));
  mix(due ? 1u : 0u);
  mix(h->reorth_due ? 1u : 0u);
  return k | 1u;  // never 0 (0 marks an empty slot)
}

// the launches of a generation up to the eigensolve set-up, eagerly or by
// replaying a captured graph; then the host counters
int front(cmaes* h) {
  set_due(h);
  const bool can_graph = h->graphs && h->st != nullptr && !h->timing && !h->kt.on;
  if (!can_graph) {
    if (int rc = phase_sample(h, nullptr)) return rc;
    if (int rc = phase_fitness(h)) return rc;
    if (int rc = phase_update_pre(h)) return rc;
    advance_counters(h);
    return 0;
  }
  const int slot = h->eig_due ? (h->reorth_due ? 2 : 1) : 0;
  const uint64_t key = front_key(h, h->eig_due);
  if (h->gx[slot] == nullptr || h->gkey[slot] != key) {
    if (h->gx[slot]) (void)hipGraphExecDestroy(h->gx[slot]);
    h->gx[slot] = nullptr;
    h->gkey[slot] = 0;
    CMX_HIP(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
    int rc = phase_sample(h, nullptr);
    if (!rc) rc = phase_fitness(h);
    if (!rc) rc = phase_update_pre(h);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(h->st, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ce != hipSuccess) return fail(CMAES_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    const hipError_t ie = hipGraphInstantiate(&h->gx[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(CMAES_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
    h->gkey[slot] = key;
  } else if (h->eig_due) {
    eigen_begin_host(h->ew);
  }
  CMX_HIP(hipGraphLaunch(h->gx[slot], h->st));
  advance_counters(h);
  return 0;
}

int read_scalars(const cmaes* h, DevScalars* s) {
  CMX_HIP(hipMemcpyAsync(s, h->sc, sizeof(*s), hipMemcpyDeviceToHost, h->st));
  CMX_HIP(hipStreamSynchronize(h->st));
  return 0;
}

// The stop bits and f_best after everything queued on the handle's stream,
// read from the mapped host copy: one stream synchronisation (none with
// sync = false, for a caller that has already waited for that work) and no
// copy.
int read_stop_best(const cmaes* h, uint32_t* stop, double* f_best, bool sync = true) {
  if (!h->allocated) {  // no generation and no state yet
    if (stop) *stop = 0;
    if (f_best) *f_best = HUGE_VAL;
    return 0;
  }
  if (sync) CMX_HIP(hipStreamSynchronize(h->st));
  if (stop) *stop = __atomic_load_n(h->hstop, __ATOMIC_ACQUIRE);
  if (f_best) {
    const uint64_t bits = __atomic_load_n(reinterpret_cast<const uint64_t*>(h->hstop + 2), __ATOMIC_ACQUIRE);
    std::memcpy(f_best, &bits, sizeof(bits));
  }
  return 0;
}

}  // namespace

extern "C" {

int cmaes_default_options(cmaes_options_t* o) {
  if (!o) return fail(CMAES_EINVAL, "null options");
  std::memset(o, 0, sizeof(*o));
  o->precision = CMAES_MIXED;
  o->eigen_interval = 0;
  o->k_max = 256;
  o->max_gens = 0;
  o->max_evals = 0;
  o->box_lo = -4.0;
  o->box_hi = 4.0;
  o->f_target = 1e-8;
  o->tol_hist_fun = 1e-12;
  o->tol_fun = 1e-12;
  o->tol_x_factor = 1e-12;
  o->max_condition = 1e14;
  o->stream = nullptr;
  return CMAES_OK;
}

const char* cmaes_last_error(void) { return g_err.c_str(); }

cmaes_t* cmaes_create(int n, int lambda, double sigma0, uint64_t seed) {
  if (n < 1) {
    set_error("n must be >= 1");
    return nullptr;
  }
  if (lambda <= 0) lambda = default_lambda(n);
  if (lambda < 2) {
    set_error("lambda must be >= 2");
    return nullptr;
  }
  if (!(sigma0 > 0.0) || !std::isfinite(sigma0)) {
    set_error("sigma0 must be positive and finite");
    return nullptr;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    set_error("no HIP device available");
    return nullptr;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(std::string("this library is built for gfx950, found ") + prop.gcnArchName);
    return nullptr;
  }
  cmaes* h = new (std::nothrow) cmaes();
  if (!h) {
    set_error("host allocation failed");
    return nullptr;
  }
  h->dev = dev;
  h->epoch = g_epoch.fetch_add(1);
  h->n = n;
  h->lam = h->lam0 = lambda;
  h->sigma0 = sigma0;
  h->seed = seed;
  h->ldn = round_up(n, 4);
  cmaes_default_options(&h->opt);
  if (hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking) != hipSuccess) {
    set_error("hipStreamCreate failed");
    delete h;
    return nullptr;
  }
  h->own_stream = true;
  for (auto& e : h->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      set_error("hipEventCreate failed");
      cmaes_destroy(h);
      return nullptr;
    }
  if (hipEventCreateWithFlags(&h->ev_stop, hipEventDisableTiming) != hipSuccess) {
    set_error("hipEventCreate failed");
    cmaes_destroy(h);
    return nullptr;
  }
  h->hp = make_params(n, lambda, 0);
  refresh_stop_params(h);
  return h;
}

void cmaes_destroy(cmaes_t* h) {
  if (!h) return;
  if (h->st) (void)hipStreamSynchronize(h->st);
  free_all(h);
  for (auto& e : h->kt.ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->ev_stop) (void)hipEventDestroy(h->ev_stop);
  if (h->own_stream && h->st) (void)hipStreamDestroy(h->st);
  delete h;
}

int cmaes_set_options(cmaes_t* h, const cmaes_options_t* o) {
  if (h) drop_graphs(h);
  if (int rc = check(h)) return rc;
  if (!o) return fail(CMAES_EINVAL, "null options");
  if (o->precision < CMAES_FP64 || o->precision > CMAES_MIXED_BF16X3)
    return fail(CMAES_EINVAL, "unknown precision");
  if (o->k_max < 1 || !(o->box_hi > o->box_lo) || o->eigen_interval < 0 || o->max_gens < 0 || o->max_evals < 0)
    return fail(CMAES_EINVAL, "invalid option value");
  if (o->variant < CMAES_VARIANT_STANDARD || o->variant > CMAES_VARIANT_SEPARABLE)
    return fail(CMAES_EINVAL, "unknown variant");
  if ((o->dev_malloc == nullptr) != (o->dev_free == nullptr))
    return fail(CMAES_EINVAL, "dev_malloc and dev_free must both be set or both be NULL");
  if (h->allocated && (o->dev_malloc != h->alloc_fn || o->dev_free != h->free_fn || o->alloc_ctx != h->alloc_ctx))
    return fail(CMAES_ESTATE, "the allocator can only change before the handle's first allocation");
  const bool started = h->allocated && (h->gen > 0 || h->restart > 0);
  const bool prec_change = (o->precision == CMAES_FP64) != (h->opt.precision == CMAES_FP64);
  const bool var_change = o->variant != h->opt.variant;
  if (started && (prec_change || var_change || o->stream != h->opt.stream))
    return fail(CMAES_ESTATE, "precision, variant and stream can only change before the first generation");
  if (h->allocated && (prec_change || var_change)) free_all(h);  // re-created lazily
  const bool box_change = o->box_lo != h->opt.box_lo || o->box_hi != h->opt.box_hi;
  if (o->stream != h->opt.stream) {
    if (h->st) (void)hipStreamSynchronize(h->st);
    if (h->own_stream && h->st) (void)hipStreamDestroy(h->st);
    if (o->stream) {
      h->st = static_cast<hipStream_t>(o->stream);
      h->own_stream = false;
    } else {
      CMX_HIP(hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking));
      h->own_stream = true;
    }
  }
  h->opt = *o;
  h->kt.st = h->st;
  h->hp = make_params(h->n, h->lam, o->eigen_interval, o->variant);
  refresh_stop_params(h);
  if (h->allocated) {
    if (int rc = alloc_pop(h)) return rc;
    if (int rc = upload_params(h)) return rc;
    if (!started && box_change) return init_descent(h, true);
    if (h->obj_kind != CMAES_OBJ_NONE) return upload_objective_derived(h);
  }
  return CMAES_OK;
}

int cmaes_get_options(const cmaes_t* h, cmaes_options_t* o) {
  if (int rc = check(h)) return rc;
  if (!o) return fail(CMAES_EINVAL, "null options");
  *o = h->opt;
  return CMAES_OK;
}

int cmaes_set_objective(cmaes_t* h, int kind, const double* R, const double* xstar) {
  if (int rc = check(h)) return rc;
  drop_graphs(h);
  if (kind < CMAES_OBJ_NONE || kind > CMAES_OBJ_RASTRIGIN) return fail(CMAES_EINVAL, "unknown objective");
  const size_t n = static_cast<size_t>(h->n);
  h->have_R = R != nullptr;
  h->have_xstar = xstar != nullptr;
  h->R_host.assign(R ? R : R, R ? R + n * n : R);
  h->xstar_host.assign(xstar ? xstar : xstar, xstar ? xstar + n : xstar);
  h->obj_kind = kind;
  if (!h->allocated) return ensure_ready(h);
  if (kind == CMAES_OBJ_NONE) return CMAES_OK;
  CMX_HIP(hipStreamSynchronize(h->st));
  return upload_objective(h);
}

int cmaes_generation(cmaes_t* h) {
  if (int rc = check(h)) return rc;
  if (h->obj_kind == CMAES_OBJ_NONE) return fail(CMAES_ESTATE, "no fused objective set (use ask/tell)");
  if (int rc = ensure_ready(h)) return rc;
  if (int rc = check_running(h)) return rc;
  if (int rc = front(h)) return rc;
  return finish_generation(h);
}

int cmaes_generation_with_z(cmaes_t* h, const double* Z) {
  if (int rc = check(h)) return rc;
  if (!Z) return fail(CMAES_EINVAL, "null Z");
  if (h->obj_kind == CMAES_OBJ_NONE) return fail(CMAES_ESTATE, "no fused objective set");
  if (int rc = ensure_ready(h)) return rc;
  if (int rc = check_running(h)) return rc;
  if (int rc = phase_sample(h, Z)) return rc;
  if (int rc = phase_fitness(h)) return rc;
  return phase_update(h);
}

}  // extern "C"

namespace {

template <typename T>
__global__ void k_points(int n, int lam, const double* __restrict__ m, const T* __restrict__ Y, int ldy,
                         const DevScalars* __restrict__ sc, double* __restrict__ X) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * lam) return;
  const int k = static_cast<int>(idx / n), i = static_cast<int>(idx % n);
  X[idx] = m[i] + sc->sigma * static_cast<double>(Y[static_cast<int64_t>(k) * ldy + i]);
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// the sampling step of an ask, then x_k = m + sigma y_k staged in dX (n * lam
// float64 device memory) and copied into the caller's X
int ask_into(cmaes* h, double* X, double* dX) {
  const int n = h->n, lam = h->lam;
  if (int rc = phase_sample(h, nullptr)) return rc;
  const int64_t total = static_cast<int64_t>(n) * lam;
  const int blocks = static_cast<int>((total + 255) / 256);
  if (h->fp64)
    k_points<double><<<blocks, 256, 0, h->st>>>(n, lam, h->m, static_cast<const double*>(h->Y), h->ldn, h->sc, dX);
  else
    k_points<float><<<blocks, 256, 0, h->st>>>(n, lam, h->m, static_cast<const float*>(h->Y), h->ldn, h->sc, dX);
  CMX_HIP(hipGetLastError());
  CMX_HIP(hipMemcpyAsync(X, dX, 8ull * total, hipMemcpyDeviceToHost, h->st));
  CMX_HIP(hipStreamSynchronize(h->st));
  h->ask_pending = true;
  return CMAES_OK;
}

// Staging memory of cmaes_ask_noalloc: a file-scope device array, one copy on
// every device the library runs on, held until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory: its device
// address on each device comes from hipGetSymbolAddress (made current device
// by device, once) and only that address is passed to kernels and copies.
constexpr size_t kScratchDoubles = size_t{1} << 20;  // 8 MiB
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on device dev (resolved on first use, with
// dev current; the caller's current device is restored)
int scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(CMAES_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    CMX_HIP(hipGetDevice(&cur));
    if (cur != dev) CMX_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr)
      return fail(CMAES_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace

extern "C" {

int cmaes_ask(cmaes_t* h, double* X) {
  if (int rc = check(h)) return rc;
  if (!X) return fail(CMAES_EINVAL, "null X");
  if (int rc = ensure_ready(h)) return rc;
  if (int rc = check_running(h)) return rc;
  if (!h->X || h->cap_lam < h->lam) {
    dev_free(h, h->X);
    if (int rc = dev_alloc(h, &h->X, 8ull * h->n * h->cap_lam)) return rc;
  }
  return ask_into(h, X, h->X);
}

int cmaes_ask_noalloc(cmaes_t* h, double* X) {
  if (int rc = check(h)) return rc;
  if (!X) return fail(CMAES_EINVAL, "null X");
  if (!h->allocated)
    return fail(CMAES_ESTATE, "cmaes_ask_noalloc needs a handle whose buffers exist (call cmaes_state, "
                              "cmaes_set_objective or cmaes_generation once first)");
  if (static_cast<size_t>(h->n) * static_cast<size_t>(h->lam) > kScratchDoubles)
    return fail(CMAES_EINVAL, "cmaes_ask_noalloc: n * lambda = " +
                                  std::to_string(static_cast<size_t>(h->n) * h->lam) + " exceeds the " +
                                  std::to_string(kScratchDoubles) + " doubles of the static staging area");
  if (int rc = check_running(h)) return rc;
  double* dX = nullptr;
  if (int rc = scratch_on(h->dev, &dX)) return rc;
  return ask_into(h, X, dX);
}

int cmaes_tell(cmaes_t* h, const double* f) {
  if (int rc = check(h)) return rc;
  if (!f) return fail(CMAES_EINVAL, "null f");
  if (!h->ask_pending) return fail(CMAES_ESTATE, "cmaes_tell without a pending cmaes_ask");
  CMX_HIP(hipMemcpyAsync(h->f, f, 8ull * h->lam, hipMemcpyHostToDevice, h->st));
  CMX_HIP(hipStreamSynchronize(h->st));  // the caller's buffer is consumed before the call returns
  h->ask_pending = false;
  return phase_update(h);
}

int cmaes_restart_ipop(cmaes_t* h) {
  if (int rc = check(h)) return rc;
  if (2 * h->K > h->opt.k_max) return fail(CMAES_EKMAX, "K would exceed K_max");
  if (int rc = ensure_ready(h)) return rc;
  CMX_HIP(hipStreamSynchronize(h->st));
  h->K *= 2;
  h->restart += 1;
  h->lam = h->K * h->lam0;
  h->hp = make_params(h->n, h->lam, h->opt.eigen_interval, h->opt.variant);
  if (int rc = alloc_pop(h)) return rc;
  if (int rc = upload_params(h)) return rc;
  return init_descent(h, false);
}

int cmaes_ipop_run(cmaes_t* h, int* descents) {
  if (int rc = check(h)) return rc;
  if (h->obj_kind == CMAES_OBJ_NONE) return fail(CMAES_ESTATE, "no fused objective set");
  int count = 1;
  for (;;) {
    const int grc = cmaes_generation(h);
    if (grc != CMAES_OK && grc != CMAES_ENUMERIC) return grc;  // ENUMERIC: stop bits are set
    DevScalars s;
    if (int rc = read_scalars(h, &s)) return rc;
    const bool budget = h->opt.max_evals > 0 && h->total_evals >= h->opt.max_evals;
    if (s.stop || budget) {
      if (s.f_best < h->opt.f_target || budget) break;
      const int rc = cmaes_restart_ipop(h);
      if (rc == CMAES_EKMAX) break;
      if (rc) return rc;
      ++count;
    }
  }
  if (descents) *descents = count;
  return CMAES_OK;
}

int cmaes_state(const cmaes_t* hc, cmaes_state_t* out) {
  if (int rc = check(hc)) return rc;
  if (!out) return fail(CMAES_EINVAL, "null state");
  cmaes_t* h = const_cast<cmaes_t*>(hc);
  if (int rc = ensure_ready(h)) return rc;
  DevScalars s;
  if (int rc = read_scalars(h, &s)) return rc;
  const int n = h->n, ldn = h->ldn;
  out->n = n;
  out->lambda = h->lam;
  out->mu = h->hp.kp.mu;
  out->restart = h->restart;
  out->gen = h->gen;
  out->evals = h->evals;
  out->total_evals = h->total_evals;
  out->sigma = s.sigma;
  out->f_best = s.f_best;
  out->stop = s.stop;
  out->kappa = h->hp.kp.kappa;
  out->eig_sweeps = s.jac_sweeps;
  out->eig_corrections = s.jac_corr;
  auto vec = [&](double* dst, const double* src) -> int {
    if (dst) CMX_HIP(hipMemcpyAsync(dst, src, 8ull * n, hipMemcpyDeviceToHost, h->st));
    return 0;
  };
  auto mat = [&](double* dst, const double* src) -> int {
    if (dst) CMX_HIP(hipMemcpy2DAsync(dst, 8ull * n, src, 8ull * ldn, 8ull * n, n, hipMemcpyDeviceToHost, h->st));
    return 0;
  };
  int rc;
  if ((rc = vec(out->m, h->m)) || (rc = vec(out->p_sigma, h->ps)) || (rc = vec(out->p_c, h->pc)) ||
      (rc = vec(out->D, h->D)) || (rc = vec(out->x_best, h->x_best)) || (rc = mat(out->C, h->C)) ||
      (rc = mat(out->B, h->B)))
    return rc;
  if (out->f) CMX_HIP(hipMemcpyAsync(out->f, h->f, 8ull * h->lam, hipMemcpyDeviceToHost, h->st));
  if (out->order) CMX_HIP(hipMemcpyAsync(out->order, h->order, 4ull * h->lam, hipMemcpyDeviceToHost, h->st));
  CMX_HIP(hipStreamSynchronize(h->st));
  return CMAES_OK;
}

int cmaes_set_state(cmaes_t* h, const cmaes_state_t* in) {
  if (int rc = check(h)) return rc;
  if (!in) return fail(CMAES_EINVAL, "null state");
  if (in->n != h->n || in->lambda != h->lam) return fail(CMAES_EINVAL, "n / lambda do not match the handle");
  if (!(in->sigma > 0.0) || in->gen < 0) return fail(CMAES_EINVAL, "sigma must be > 0 and gen >= 0");
  if (int rc = ensure_ready(h)) return rc;
  const int n = h->n, ldn = h->ldn;
  DevScalars s;
  CMX_HIP(hipMemcpyAsync(&s, h->sc, sizeof(s), hipMemcpyDeviceToHost, h->st));
  CMX_HIP(hipStreamSynchronize(h->st));  // also: nothing in flight still writes the state
  s.sigma = in->sigma;
  s.gen = in->gen;
  s.stop = 0;
  s.hist_count = 0;
  s.eig_ok = 1;
  // every copy below is ordered on the handle's stream and has completed
  // before the call returns (the caller's buffers are then no longer read)
  CMX_HIP(hipMemcpyAsync(h->sc, &s, sizeof(s), hipMemcpyHostToDevice, h->st));
  h->gen = in->gen;
  auto vec_in = [&](double* dst, const double* src) -> int {
    if (src) CMX_HIP(hipMemcpyAsync(dst, src, 8ull * n, hipMemcpyHostToDevice, h->st));
    return 0;
  };
  int rc;
  if ((rc = vec_in(h->m, in->m)) || (rc = vec_in(h->ps, in->p_sigma)) || (rc = vec_in(h->pc, in->p_c)) ||
      (rc = vec_in(h->D, in->D)))
    return rc;
  if (in->C)
    CMX_HIP(hipMemcpy2DAsync(h->C, 8ull * ldn, in->C, 8ull * n, 8ull * n, n, hipMemcpyHostToDevice, h->st));
  if (in->B) {
    CMX_HIP(hipMemcpy2DAsync(h->B, 8ull * ldn, in->B, 8ull * n, 8ull * n, n, hipMemcpyHostToDevice, h->st));
    CMX_HIP(hipMemsetAsync(h->ew.gctl, 0, 4ull * GC_WORDS, h->st));  // no previous solve
    h->reorth_sweeps = 0;  // taken as orthogonal
    h->eig_uncounted = false;
    h->ew.last_sweeps = 0;
    h->ew.last_closed = false;
  }
  if (in->B || in->D) {
    // B D in the sampling precision
    std::vector<double> Bh(static_cast<size_t>(n) * n), Dh(n);
    CMX_HIP(hipMemcpy2DAsync(Bh.data(), 8ull * n, h->B, 8ull * ldn, 8ull * n, n, hipMemcpyDeviceToHost, h->st));
    CMX_HIP(hipMemcpyAsync(Dh.data(), h->D, 8ull * n, hipMemcpyDeviceToHost, h->st));
    CMX_HIP(hipStreamSynchronize(h->st));
    for (int c = 0; c < n; ++c)
      for (int r = 0; r < n; ++r) Bh[static_cast<size_t>(c) * n + r] *= Dh[c];
    CMX_HIP(hipMemcpy2DAsync(h->ew.T, 8ull * ldn, Bh.data(), 8ull * n, 8ull * n, n, hipMemcpyHostToDevice, h->st));
    CMX_HIP(launch_to_precision(h->st, h->fp64, h->ew.T, ldn, h->BD, ldn, n, n));
  }
  CMX_HIP(hipStreamSynchronize(h->st));
  *h->hstop = 0;  // the stop bits were cleared
  *host_fbest(h) = s.f_best;
  h->stop_pending = false;
  h->ask_pending = false;
  return CMAES_OK;
}

int cmaes_enable_timing(cmaes_t* h, int on) {
  if (int rc = check(h)) return rc;
  h->timing = on != 0;
  return CMAES_OK;
}

int cmaes_enable_graphs(cmaes_t* h, int on) {
  if (int rc = check(h)) return rc;
  h->graphs = on != 0;
  drop_graphs(h);
  return CMAES_OK;
}

int cmaes_set_eigen_correction(cmaes_t* h, int on, double max_angle_norm) {
  if (int rc = check(h)) return rc;
  if (!(max_angle_norm >= 0.0 && max_angle_norm <= 2e-3)) return fail(CMAES_EINVAL, "max_angle_norm not in [0, 2e-3]");
  if (max_angle_norm != h->ew.corr_max_theta) eigen_drop_graphs(h->ew);  // captured as a kernel argument
  h->ew.correct_on = on != 0;
  h->ew.corr_max_theta = max_angle_norm;
  h->ew.last_closed = false;
  return CMAES_OK;
}

int cmaes_enable_kernel_timing(cmaes_t* h, int on) {
  if (int rc = check(h)) return rc;
  if (on && !h->kt.ev[0]) {
    for (auto& e : h->kt.ev) CMX_HIP(hipEventCreate(&e));
  }
  h->kt.on = on != 0;
  h->kt.st = h->st;
  h->kt.used = 0;
  for (int i = 0; i < KID_COUNT; ++i) {
    h->kt.total_us[i] = 0.0;
    h->kt.calls[i] = 0;
  }
  return CMAES_OK;
}

int cmaes_kernel_times(const cmaes_t* h, double* total_us, int64_t* calls) {
  if (int rc = check(h)) return rc;
  if (!total_us || !calls) return fail(CMAES_EINVAL, "null output");
  for (int i = 0; i < KID_COUNT; ++i) {
    total_us[i] = h->kt.total_us[i];
    calls[i] = h->kt.calls[i];
  }
  return CMAES_OK;
}

int cmaes_phase_times(const cmaes_t* h, double* out) {
  if (int rc = check(h)) return rc;
  if (!out) return fail(CMAES_EINVAL, "null output");
  for (int i = 0; i < CMAES_NUM_PHASES; ++i) out[i] = h->phase_us[i];
  return CMAES_OK;
}

int cmaes_gemm_config_count(void) { return kG32NumConfigs; }

int cmaes_gemm_config_info(int cfg, int32_t* bm, int32_t* bn, int32_t* bk) {
  if (cfg < 0 || cfg >= kG32NumConfigs) return fail(CMAES_EINVAL, "no such tile configuration");
  if (bm) *bm = kG32Configs[cfg].bm;
  if (bn) *bn = kG32Configs[cfg].bn;
  if (bk) *bk = kG32Configs[cfg].bk;
  return CMAES_OK;
}

int cmaes_set_gemm_config(cmaes_t* h, int site, int cfg) {
  if (int rc = check(h)) return rc;
  if (site < 0 || site >= G32_NUM_SITES) return fail(CMAES_EINVAL, "no such GEMM site");
  if (!g32_config_valid(cfg, site)) return fail(CMAES_EINVAL, "tile configuration not available at this site");
  h->gcfg[site] = cfg;
  return CMAES_OK;
}

int cmaes_get_gemm_config(const cmaes_t* h, int site, int32_t* cfg) {
  if (int rc = check(h)) return rc;
  if (site < 0 || site >= G32_NUM_SITES || !cfg) return fail(CMAES_EINVAL, "bad site or null output");
  *cfg = h->gcfg[site];
  return CMAES_OK;
}

int cmaes_autotune(cmaes_t* h, int reps, double* us, int32_t* chosen) {
  if (int rc = check(h)) return rc;
  if (reps < 1) return fail(CMAES_EINVAL, "reps must be positive");
  if (h->ask_pending) return fail(CMAES_ESTATE, "autotune between ask and tell");
  if (int rc = ensure_ready(h)) return rc;
  if (us)
    for (int i = 0; i < G32_NUM_SITES * kG32NumConfigs; ++i) us[i] = -1.0;
  if (!h->fp64) {
    const int n = h->n, lam = h->lam, ldn = h->ldn, mu = h->hp.kp.mu;
    // operands with the next generation's statistics: its own normals and the
    // current B D; the next generation redraws Z and rewrites Y, Ysel
    CMX_HIP(launch_normals(h->st, h->Z, false, ldn, n, lam, h->seed, static_cast<uint32_t>(h->restart), h->sc));
    CMX_HIP(hipMemcpyAsync(h->Y, h->Z, 4ull * ldn * lam, hipMemcpyDeviceToDevice, h->st));
    CMX_HIP(hipMemcpyAsync(h->Ysel, h->Z, 4ull * ldn * mu, hipMemcpyDeviceToDevice, h->st));
    hipEvent_t e0, e1;
    CMX_HIP(hipEventCreate(&e0));
    CMX_HIP(hipEventCreate(&e1));
    const G32FitArgs ga{h->obj_kind, h->d, static_cast<const float*>(h->coef), h->sc};
    // the covariance site is timed with its epilogue, which then updates this
    // scratch matrix instead of C (tiles differ in how many partials it sums)
    double* cscratch = nullptr;
    int rc = dev_alloc(h, &cscratch, 8ull * ldn * n);
    for (int site = 0; site < G32_NUM_SITES && rc == CMAES_OK; ++site) {
      if (site == G32_SAMPLE && h->opt.precision == CMAES_MIXED_BF16X3) continue;
      if (site == G32_FITNESS && !(h->have_R && h->obj_kind != CMAES_OBJ_NONE)) continue;
      double best = HUGE_VAL;
      for (int c = 0; c < kG32NumConfigs && rc == CMAES_OK; ++c) {
        if (!g32_config_valid(c, site)) continue;
        auto launch = [&]() -> hipError_t {
          if (site == G32_SAMPLE)
            return g32_gemm(h->st, c, site, n, lam, n, static_cast<const float*>(h->BD), ldn,
                            static_cast<const float*>(h->Z), ldn, h->Y, ldn, nullptr);
          if (site == G32_FITNESS)
            return g32_gemm(h->st, c, site, n, lam, n, static_cast<const float*>(h->Rt), ldn,
                            static_cast<const float*>(h->Y), ldn, h->partial, lam, &ga);
          return g32_syrk(h->st, c, n, mu, static_cast<const float*>(h->Ysel), nullptr, ldn,
                          static_cast<float*>(h->syrk_work),
                          cscratch, ldn, h->pc, 0.0, 0.0, h->sc, false, nullptr);
        };
        hipError_t e = launch();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, h->st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, h->st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          rc = fail(CMAES_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
          break;
        }
        const double t = 1e3 * ms / reps;
        if (us) us[site * kG32NumConfigs + c] = t;
        if (t < best) {
          best = t;
          h->gcfg[site] = c;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(h->st);
    dev_free(h, cscratch);
    if (rc) return rc;
  }
  if (chosen)
    for (int i = 0; i < G32_NUM_SITES; ++i) chosen[i] = h->gcfg[i];
  return CMAES_OK;
}

int cmaes_device_arch(char* buf, int len) {
  if (!buf || len < 1) return fail(CMAES_EINVAL, "null or empty buffer");
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
    return fail(CMAES_EDEVICE, "no HIP device");
  std::snprintf(buf, static_cast<size_t>(len), "%s", p.gcnArchName);
  return CMAES_OK;
}

int cmaes_syrk_plan(int cfg, int n, int K, int32_t* tiles, int32_t* kspan, int32_t* splits) {
  if (!g32_config_valid(cfg, G32_SYRK) || n < 1 || K < 1)
    return fail(CMAES_EINVAL, "cfg must be a square tile configuration, n and K >= 1");
  int ntl = 0, sp = 0, ks = 0;
  size_t we = 0;
  syrk32_plan(cfg, n, K, &ntl, &sp, &ks, &we);
  if (tiles) *tiles = ntl;
  if (kspan) *kspan = ks;
  if (splits) *splits = sp;
  return CMAES_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched concurrent descents (K-Distributed, Sec. 3.2.3): every instance is a
// full handle with its own stream, so the hardware interleaves the kernels of
// all instances; a batch generation queues every instance up to its
// eigensolve, then advances all sweeps in lockstep with one host
// synchronisation per sweep for the whole batch.  An instance whose stop
// tests fire is restarted with the same population size (restart-on-finish).

namespace {

// The eigensolves of a set of descents stepped together (the batch of
// concurrent descents, the K-Replicated tree): one grouped solve on a stream
// of the set's own, which waits for every due descent's front and which the
// descents' stop tests wait for.
// the grouped front's tables (see GFront): the descents, the four float64
// products per descent (re-orthogonalisation B^T B and B G, warm start C B
// and B^T T), and the workgroup offsets of every step
constexpr int kFrontMM = 4;  // products: RO_G, RO_T, CB, BT
struct FrontTables {
  void* dmem = nullptr;  // device copy: GFront[cap], GDgemm[kFrontMM][cap], offsets
  int cap = 0, count = 0;
  std::vector<GFront> tab;
  std::vector<GDgemm> mm;   // kFrontMM x count
  std::vector<int> off;     // GF_KINDS x (count + 1)
  std::vector<int> offmm;   // kFrontMM x 2 x (count + 1): products, adds
  std::vector<uint64_t> keys;
  int cfg[G32_NUM_SITES] = {0, 0, 0};
};

struct LockstepGroup {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  GroupEig ge;
  std::vector<cmaes*> members;  // the descents the table was built for
  std::vector<uint64_t> epochs;  // their buffer epochs then
  std::vector<hipEvent_t> ev;    // per member: the end of its front
  std::vector<int> sweeps;
  FrontTables ft;
  std::vector<cmaes*> fmembers;  // the descents the front tables were built for
  // the last lockstep generation ended with the host waiting for the group,
  // so every member's stream was idle and its stop copy current on return
  bool synced = false;
};

int group_init(LockstepGroup& g) {
  CMX_HIP(hipStreamCreateWithFlags(&g.st, hipStreamNonBlocking));
  CMX_HIP(hipEventCreateWithFlags(&g.done, hipEventDisableTiming));
  return 0;
}

void group_destroy(LockstepGroup& g) {
  if (g.st) (void)hipStreamSynchronize(g.st);
  group_eig_release(g.ge);
  if (g.ft.dmem) (void)hipFree(g.ft.dmem);
  for (auto e : g.ev)
    if (e) (void)hipEventDestroy(e);
  g.ev.clear();
  if (g.done) (void)hipEventDestroy(g.done);
  if (g.st) (void)hipStreamDestroy(g.st);
  g = LockstepGroup{};
}

GEigDesc eig_desc(cmaes* h) {
  GEigDesc e{};
  EigWork& w = h->ew;
  e.A = w.A;
  e.A2 = w.A2;
  e.V = w.V;
  e.Q = w.Q;
  e.Q2 = w.Q2;
  e.part = w.part;
  e.scale = w.scale;
  e.C = h->C;
  e.ldc = h->ldn;
  e.status = w.status;
  e.ctl = w.gctl;
  e.B = h->B;
  e.ldb = h->ldn;
  e.D = h->D;
  e.BD = h->BD;
  e.ldbd = h->ldn;
  e.bd64 = h->fp64 ? 1 : 0;
  e.evals = w.evals;
  e.perm = w.perm;
  e.sign = w.sign;
  e.sc = h->sc;
  e.n = h->n;
  e.N = w.N;
  return e;
}

}  // namespace

struct cmaes_batch {
  std::vector<cmaes*> inst;
  std::vector<int32_t> restarts;
  LockstepGroup grp;
};

namespace {

int restart_same_lambda(cmaes* h) {
  CMX_HIP(hipStreamSynchronize(h->st));
  h->restart += 1;
  return init_descent(h, false);
}

// whether a set of descents can run the grouped front: mixed precision with
// float32 sampling, a rotated fused objective, the same GEMM tiles, no timers
bool front_groupable(const std::vector<cmaes*>& hs) {
  for (cmaes* h : hs) {
    if (h->fp64 || h->opt.precision != CMAES_MIXED || h->opt.variant != CMAES_VARIANT_STANDARD || !h->have_R ||
        h->obj_kind == CMAES_OBJ_NONE || h->timing || h->kt.on)
      return false;
    for (int s = 0; s < G32_NUM_SITES; ++s)
      if (h->gcfg[s] != hs[0]->gcfg[s]) return false;
  }
  return !hs.empty();
}

uint64_t front_member_key(const cmaes* h) {
  uint64_t k = h->epoch;
  k = k * 0x100000001B3ull + static_cast<uint64_t>(h->lam);
  k = k * 0x100000001B3ull + static_cast<uint64_t>(h->restart);
  return k;
}

GDgemm dgemm_desc(const double* A, int lda, const double* B, int ldb, double* C, int ldc, double* W, int ldw, int n) {
  // launch_dgemm_ksplit's plan: two half-k products while the product has at
  // most one 64 x 64 tile per CU
  const int tiles = ceil_div(n, 64) * ceil_div(n, 64);
  const int K0 = round_up(ceil_div(n, 2), 16);
  GDgemm d{A, lda, B, ldb, C, ldc, W, ldw, n, K0, (K0 < n && tiles <= 256) ? 1 : 0};
  return d;
}

int build_front_tables(LockstepGroup& g, const std::vector<cmaes*>& hs) {
  FrontTables& ft = g.ft;
  const int count = static_cast<int>(hs.size());
  bool same = g.fmembers == hs && static_cast<int>(ft.keys.size()) == count;
  for (int i = 0; same && i < count; ++i) same = ft.keys[i] == front_member_key(hs[i]);
  for (int s = 0; same && s < G32_NUM_SITES; ++s) same = ft.cfg[s] == hs[0]->gcfg[s];
  if (same) return 0;
  ft.tab.assign(count, GFront{});
  ft.mm.assign(static_cast<size_t>(kFrontMM) * count, GDgemm{});
  ft.off.assign(static_cast<size_t>(GF_KINDS) * (count + 1), 0);
  ft.offmm.assign(static_cast<size_t>(kFrontMM) * 2 * (count + 1), 0);
  for (int s = 0; s < G32_NUM_SITES; ++s) ft.cfg[s] = hs[0]->gcfg[s];
  for (int i = 0; i < count; ++i) {
    cmaes* h = hs[i];
    const int n = h->n, lam = h->lam, mu = h->hp.kp.mu, ldn = h->ldn, N = h->ew.N;
    GFront& e = ft.tab[i];
    e.n = n;
    e.lam = lam;
    e.mu = mu;
    e.ldn = ldn;
    e.N = N;
    e.k0 = static_cast<uint32_t>(h->seed);
    e.k1 = static_cast<uint32_t>(h->seed >> 32);
    e.restart = static_cast<uint32_t>(h->restart);
    e.sc = h->sc;
    e.hstop = h->dstop;
    e.BD = static_cast<const float*>(h->BD);
    e.Z = static_cast<float*>(h->Z);
    e.Y = static_cast<float*>(h->Y);
    e.Rd = h->Rd;
    e.m = h->m;
    e.xstar = h->have_xstar ? h->xstar : nullptr;
    e.u = h->u;
    e.part_bz = h->part_bz;
    e.d = h->d;
    e.kind = h->obj_kind;
    e.fit_tiles = g32_row_tiles(ft.cfg[G32_FITNESS], n);
    e.Rt = static_cast<const float*>(h->Rt);
    e.coef = static_cast<const float*>(h->coef);
    e.partial = static_cast<float*>(h->partial);
    e.f = h->f;
    e.rank_work = h->rank_work;
    e.order = h->order;
    e.x_best = h->x_best;
    e.hist = h->hist;
    e.hist_len = h->sp.hist_len;
    e.w = h->w;
    e.sqrtw = h->sqrtw;
    e.Ysel = static_cast<float*>(h->Ysel);
    e.part_yw = h->part_yw;
    e.part_zw = h->part_zw;
    e.yw = h->yw;
    e.zw = h->zw;
    e.B = h->B;
    e.D = h->D;
    e.ps = h->ps;
    e.pc = h->pc;
    e.kp = h->hp.kp;
    e.syrk_work = static_cast<float*>(h->syrk_work);
    e.C = h->C;
    {
      size_t we;
      syrk32_plan(ft.cfg[G32_SYRK], n, mu, &e.syrk_ntl, &e.syrk_splits, &e.syrk_kspan, &we);
    }
    e.V = h->ew.V;
    e.A = h->ew.A;
    e.A2 = h->ew.A2;
    e.T = h->ew.T;
    e.epart = h->ew.part;
    e.scale = h->ew.scale;
    e.dflags = h->ew.dflags;
    e.gctl = h->ew.gctl;
    e.sp = h->sp;
    // the products of the re-orthogonalisation and of the warm start
    ft.mm[0 * count + i] = dgemm_desc(h->B, ldn, h->B, ldn, h->ew.A2, N, h->ew.X2, N, n);      // G = B^T B
    ft.mm[1 * count + i] = dgemm_desc(h->B, ldn, h->ew.A2, N, h->ew.T, ldn, h->ew.X2, N, n);   // T = B G
    ft.mm[2 * count + i] = dgemm_desc(h->C, ldn, h->B, ldn, h->ew.T, ldn, h->ew.X2, N, n);     // T = C B
    ft.mm[3 * count + i] = dgemm_desc(h->B, ldn, h->ew.T, ldn, h->ew.A, N, h->ew.X2, N, n);    // A = B^T T
    // workgroups per descent of every step
    int wgs[GF_KINDS] = {};
    const int nb256 = ceil_div(n, 256);
    wgs[GF_NORMALS] = static_cast<int>((static_cast<int64_t>((n + 3) / 4) * lam + 255) / 256);
    wgs[GF_SAMPLE] = g32_tiles(ft.cfg[G32_SAMPLE], n, lam);
    wgs[GF_SUB] = nb256;
    wgs[GF_RMATVEC] = nb256 * ceil_div(n, 64);
    wgs[GF_RVEC] = nb256;
    wgs[GF_FITNESS] = g32_tiles(ft.cfg[G32_FITNESS], n, lam);
    wgs[GF_FREDUCE] = ceil_div(lam, 256);
    wgs[GF_RANK] = rank_chunks(lam);
    wgs[GF_MERGE] = rank_merge_wgs(lam);
    wgs[GF_SCATTER] = rank_chunks(lam);
    wgs[GF_BEST] = 1;
    wgs[GF_RECOMB] = nb256 * ceil_div(mu, 64);
    wgs[GF_REDYZ] = nb256;
    wgs[GF_BMATVEC] = nb256 * ceil_div(n, 64);
    wgs[GF_VECUPD] = 1;
    syrk32_group_wgs(ft.cfg[G32_SYRK], n, mu, &wgs[GF_SYRK], &wgs[GF_SYRKEPI]);
    wgs[GF_INIT] = static_cast<int>((static_cast<int64_t>(N) * N + 255) / 256);
    wgs[GF_OFFCOLS] = n;
    wgs[GF_OFFFIN] = 1;
    wgs[GF_POLAR] = static_cast<int>((static_cast<int64_t>(n) * n + 255) / 256);
    wgs[GF_STOP] = 1;
    for (int k = 0; k < GF_KINDS; ++k) ft.off[k * (count + 1) + i + 1] = ft.off[k * (count + 1) + i] + wgs[k];
    for (int q = 0; q < kFrontMM; ++q) {
      const GDgemm& d = ft.mm[q * count + i];
      const int tiles = ceil_div(n, 64) * ceil_div(n, 64);
      const int prod = d.split ? 2 * tiles : tiles, add = d.split ? nb256 * n : 0;
      int* o = ft.offmm.data() + static_cast<size_t>(q) * 2 * (count + 1);
      o[i + 1] = o[i] + prod;
      o[(count + 1) + i + 1] = o[(count + 1) + i] + add;
    }
  }
  if (ft.cap < count) {
    if (ft.dmem) (void)hipFree(ft.dmem);
    ft.dmem = nullptr;
    const size_t bytes = sizeof(GFront) * kGroupMax + sizeof(GDgemm) * kFrontMM * kGroupMax +
                         sizeof(int) * (GF_KINDS + 2 * kFrontMM) * (kGroupMax + 1);
    if (hipMalloc(&ft.dmem, bytes) != hipSuccess) return fail(CMAES_ENOMEM, "grouped front: hipMalloc failed");
    ft.cap = kGroupMax;
  }
  char* base = static_cast<char*>(ft.dmem);
  CMX_HIP(hipMemcpyAsync(base, ft.tab.data(), sizeof(GFront) * count, hipMemcpyHostToDevice, g.st));
  for (int q = 0; q < kFrontMM; ++q)
    CMX_HIP(hipMemcpyAsync(base + sizeof(GFront) * kGroupMax + sizeof(GDgemm) * q * kGroupMax,
                           ft.mm.data() + static_cast<size_t>(q) * count, sizeof(GDgemm) * count,
                           hipMemcpyHostToDevice, g.st));
  char* offb = base + sizeof(GFront) * kGroupMax + sizeof(GDgemm) * kFrontMM * kGroupMax;
  CMX_HIP(hipMemcpyAsync(offb, ft.off.data(), sizeof(int) * ft.off.size(), hipMemcpyHostToDevice, g.st));
  CMX_HIP(hipMemcpyAsync(offb + sizeof(int) * GF_KINDS * (count + 1), ft.offmm.data(),
                         sizeof(int) * ft.offmm.size(), hipMemcpyHostToDevice, g.st));
  CMX_HIP(hipStreamSynchronize(g.st));  // the host vectors are consumed
  ft.count = count;
  ft.keys.clear();
  for (cmaes* h : hs) ft.keys.push_back(front_member_key(h));
  g.fmembers = hs;
  return 0;
}

// the fixed part of one generation of every descent, one launch per step for
// all of them, on the group's stream (the per-descent equivalent is front())
int grouped_front(LockstepGroup& g, const std::vector<cmaes*>& hs, const GroupDueMask& due,
                  const GroupDueMask& reorth, bool any_due, bool any_reorth) {
  FrontTables& ft = g.ft;
  const int count = ft.count;
  const char* base = static_cast<const char*>(ft.dmem);
  const GFront* tab = reinterpret_cast<const GFront*>(base);
  const GDgemm* mm = reinterpret_cast<const GDgemm*>(base + sizeof(GFront) * kGroupMax);
  const int* offd = reinterpret_cast<const int*>(base + sizeof(GFront) * kGroupMax +
                                                 sizeof(GDgemm) * kFrontMM * kGroupMax);
  auto off = [&](int k) { return offd + k * (count + 1); };
  auto wgs = [&](int k) { return ft.off[k * (count + 1) + count]; };
  const int* offmm = offd + GF_KINDS * (count + 1);
  auto moff = [&](int q, int a) { return offmm + (q * 2 + a) * (count + 1); };
  auto mwgs = [&](int q, int a) { return ft.offmm[(q * 2 + a) * (count + 1) + count]; };
  hipStream_t st = g.st;
  (void)hs;
  CMX_HIP(launch_group_normals(st, tab, off(GF_NORMALS), count, wgs(GF_NORMALS)));
  CMX_HIP(launch_group_g32(st, ft.cfg[G32_SAMPLE], G32_SAMPLE, tab, off(GF_SAMPLE), count, wgs(GF_SAMPLE)));
  for (int k : {GF_SUB, GF_RMATVEC, GF_RVEC})
    CMX_HIP(launch_group_update(st, k, tab, off(k), count, wgs(k), nullptr));
  CMX_HIP(launch_group_g32(st, ft.cfg[G32_FITNESS], G32_FITNESS, tab, off(GF_FITNESS), count, wgs(GF_FITNESS)));
  CMX_HIP(launch_group_fitness_reduce(st, tab, off(GF_FREDUCE), count, wgs(GF_FREDUCE)));
  for (int k : {GF_RANK, GF_MERGE, GF_SCATTER, GF_BEST, GF_RECOMB, GF_REDYZ, GF_BMATVEC, GF_VECUPD})
    CMX_HIP(launch_group_update(st, k, tab, off(k), count, wgs(k), nullptr));
  CMX_HIP(launch_group_syrk(st, ft.cfg[G32_SYRK], tab, off(GF_SYRK), wgs(GF_SYRK), off(GF_SYRKEPI), wgs(GF_SYRKEPI),
                            count));
  if (any_reorth) {
    CMX_HIP(launch_group_dgemm(st, true, mm + 0 * kGroupMax, moff(0, 0), mwgs(0, 0), moff(0, 1), mwgs(0, 1), count,
                               reorth));
    CMX_HIP(launch_group_dgemm(st, false, mm + 1 * kGroupMax, moff(1, 0), mwgs(1, 0), moff(1, 1), mwgs(1, 1), count,
                               reorth));
    CMX_HIP(launch_group_update(st, GF_POLAR, tab, off(GF_POLAR), count, wgs(GF_POLAR), &reorth));
  }
  // warm starts of the due descents, except those whose single-workgroup
  // solve forms its own
  GroupDueMask begin = due;
  bool any_begin = false;
  for (int i = 0; i < count; ++i)
    if (due_mask_bit(due, i)) {
      if (hs[i]->ew.N == kWholeSolveN)
        begin.w[i >> 5] &= ~(1u << (i & 31));
      else
        any_begin = true;
    }
  if (any_due && any_begin) {
    CMX_HIP(launch_group_eigen_begin(st, GF_INIT, tab, off(GF_INIT), count, wgs(GF_INIT), begin));
    CMX_HIP(launch_group_dgemm(st, false, mm + 2 * kGroupMax, moff(2, 0), mwgs(2, 0), moff(2, 1), mwgs(2, 1), count,
                               begin));
    CMX_HIP(launch_group_dgemm(st, true, mm + 3 * kGroupMax, moff(3, 0), mwgs(3, 0), moff(3, 1), mwgs(3, 1), count,
                               begin));
    CMX_HIP(launch_group_eigen_begin(st, GF_OFFCOLS, tab, off(GF_OFFCOLS), count, wgs(GF_OFFCOLS), begin));
    CMX_HIP(launch_group_eigen_begin(st, GF_OFFFIN, tab, off(GF_OFFFIN), count, wgs(GF_OFFFIN), begin));
  }
  return 0;
}

// one generation of every handle: all fronts queued first (each on its own
// stream, the warm start of a due eigensolve included), then one grouped
// eigensolve of every due handle (one launch per round for all of them,
// convergence decided on the device), then the stop tests
int lockstep_generation(LockstepGroup& g, const std::vector<cmaes*>& hs) {
  for (cmaes* h : hs)
    if (h->obj_kind == CMAES_OBJ_NONE) return fail(CMAES_ESTATE, "every instance needs a fused objective");
  const int count = static_cast<int>(hs.size());
  if (count > kGroupMax) return fail(CMAES_EINVAL, "too many descents in one lockstep group");
  for (cmaes* h : hs)
    if (int rc = ensure_ready(h)) return rc;
  const bool grouped = front_groupable(hs);
  GroupDueMask due{}, reorth{};
  bool any_reorth = false;
  if (grouped) {
    if (int rc = build_front_tables(g, hs)) return rc;
    // every descent's earlier work (a restart, a state upload) is ordered
    // before the grouped launches
    while (static_cast<int>(g.ev.size()) < count) {
      hipEvent_t e = nullptr;
      CMX_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      g.ev.push_back(e);
    }
    for (int i = 0; i < count; ++i) {
      // a descent's stream is usually idle here (the calls between
      // generations wait for their own work); only one with work still
      // queued needs the event
      const hipError_t q = hipStreamQuery(hs[i]->st);
      (void)hipGetLastError();  // a not-ready query is not an error of the next launch
      if (q == hipSuccess) continue;
      CMX_HIP(hipEventRecord(g.ev[i], hs[i]->st));
      CMX_HIP(hipStreamWaitEvent(g.st, g.ev[i], 0));
    }
    for (int i = 0; i < count; ++i) {
      set_due(hs[i]);
      if (hs[i]->eig_due) due.w[i >> 5] |= 1u << (i & 31);
      if (hs[i]->reorth_due) {
        reorth.w[i >> 5] |= 1u << (i & 31);
        any_reorth = true;
      }
    }
  } else {
    for (cmaes* h : hs)
      if (int rc = front(h)) return rc;
  }
  int ahead = 0;
  bool any = false;
  for (int i = 0; i < count; ++i)
    if (hs[i]->eig_due) {
      due.w[i >> 5] |= 1u << (i & 31);
      any = true;
      // the run of sweeps a descent makes before its first convergence test
      const int last = hs[i]->ew.last_sweeps;
      ahead = std::max(ahead, last >= 2 ? last - 1 : 0);
    }
  if (grouped) {
    if (int rc = grouped_front(g, hs, due, reorth, any, any_reorth)) return rc;
    for (cmaes* h : hs) {
      advance_counters(h);
      if (h->eig_due) eigen_begin_host(h->ew);
    }
  }
  if (any) {
    bool same = g.members == hs && static_cast<int>(g.epochs.size()) == count;
    for (int i = 0; same && i < count; ++i) same = g.epochs[i] == hs[i]->epoch;
    if (!same) {
      std::vector<GEigDesc> descs;
      for (cmaes* h : hs) descs.push_back(eig_desc(h));
      if (int rc = group_eig_build(g.st, g.ge, descs)) return rc;
      g.members = hs;
      g.epochs.clear();
      for (cmaes* h : hs) g.epochs.push_back(h->epoch);
    }
    while (static_cast<int>(g.ev.size()) < count) {
      hipEvent_t e = nullptr;
      CMX_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      g.ev.push_back(e);
    }
    if (!grouped)
      for (int i = 0; i < count; ++i)
        if (hs[i]->eig_due) {
          CMX_HIP(hipEventRecord(g.ev[i], hs[i]->st));
          CMX_HIP(hipStreamWaitEvent(g.st, g.ev[i], 0));
        }
    g.sweeps.assign(count, 0);
    if (int rc = group_eig_solve(g.st, g.ge, due, 40, ahead, g.sweeps.data(), nullptr)) return rc;
    if (!grouped) CMX_HIP(hipEventRecord(g.done, g.st));
    for (int i = 0; i < count; ++i)
      if (hs[i]->eig_due) {
        cmaes* h = hs[i];
        if (!grouped) CMX_HIP(hipStreamWaitEvent(h->st, g.done, 0));
        h->ew.sweeps = g.sweeps[i];
        h->ew.corrections = 0;
        h->ew.last_sweeps = g.sweeps[i];
        h->ew.last_closed = false;
        h->ew.pending = false;
      }
  }
  if (grouped) {
    // the stop tests of every descent (they also write its mapped copy of
    // the stop bits and f_best)
    const FrontTables& ft = g.ft;
    const char* base = static_cast<const char*>(ft.dmem);
    const int* offd = reinterpret_cast<const int*>(base + sizeof(GFront) * kGroupMax +
                                                   sizeof(GDgemm) * kFrontMM * kGroupMax);
    CMX_HIP(launch_group_update(g.st, GF_STOP, reinterpret_cast<const GFront*>(base), offd + GF_STOP * (count + 1),
                                count, ft.off[GF_STOP * (count + 1) + count], nullptr));
    // the host waits for the group (the callers read every descent's stop
    // bits next anyway), so later work on a descent's own stream is ordered
    // after the group without an event wait per stream
    CMX_HIP(hipStreamSynchronize(g.st));
    for (cmaes* h : hs) h->stop_pending = false;
    g.synced = true;
    return 0;
  }
  g.synced = false;
  for (cmaes* h : hs)
    if (int rc = phase_update_post(h)) return rc;
  return 0;
}

int batch_check(const cmaes_batch* b, int k) {
  if (!b) return fail(CMAES_EINVAL, "null batch");
  if (k < 0 || k >= static_cast<int>(b->inst.size())) return fail(CMAES_EINVAL, "instance index out of range");
  return 0;
}

}  // namespace

extern "C" {

cmaes_batch_t* cmaes_batch_create(int count, const int* n, const int* lambda, const double* sigma0,
                                  const uint64_t* seed) {
  if (count < 1 || count > 1024 || !n || !lambda || !sigma0 || !seed) {
    set_error("cmaes_batch_create: need 1..1024 instances and non-null size arrays");
    return nullptr;
  }
  cmaes_batch* b = new (std::nothrow) cmaes_batch();
  if (!b) {
    set_error("host allocation failed");
    return nullptr;
  }
  if (group_init(b->grp)) {
    const std::string why = g_err;
    cmaes_batch_destroy(b);
    set_error(why);
    return nullptr;
  }
  for (int k = 0; k < count; ++k) {
    cmaes* h = cmaes_create(n[k], lambda[k], sigma0[k], seed[k]);
    if (!h) {
      const std::string why = g_err;
      cmaes_batch_destroy(b);
      set_error("instance " + std::to_string(k) + ": " + why);
      return nullptr;
    }
    b->inst.push_back(h);
    b->restarts.push_back(0);
  }
  return b;
}

void cmaes_batch_destroy(cmaes_batch_t* b) {
  if (!b) return;
  group_destroy(b->grp);
  for (cmaes* h : b->inst) cmaes_destroy(h);
  delete b;
}

int cmaes_batch_count(const cmaes_batch_t* b) {
  if (!b) return fail(CMAES_EINVAL, "null batch");
  return static_cast<int>(b->inst.size());
}

int cmaes_batch_set_options(cmaes_batch_t* b, const cmaes_options_t* opt) {
  if (!b) return fail(CMAES_EINVAL, "null batch");
  if (!opt) return fail(CMAES_EINVAL, "null options");
  cmaes_options_t o = *opt;
  for (cmaes* h : b->inst) {
    o.stream = h->opt.stream;  // every instance keeps its own stream
    if (int rc = cmaes_set_options(h, &o)) return rc;
  }
  return CMAES_OK;
}

int cmaes_batch_enable_graphs(cmaes_batch_t* b, int on) {
  if (!b) return fail(CMAES_EINVAL, "null batch");
  for (cmaes* h : b->inst)
    if (int rc = cmaes_enable_graphs(h, on)) return rc;
  return CMAES_OK;
}

int cmaes_batch_set_objective(cmaes_batch_t* b, int k, int kind, const double* R, const double* xstar) {
  if (int rc = batch_check(b, k)) return rc;
  return cmaes_set_objective(b->inst[k], kind, R, xstar);
}

int cmaes_batch_generation(cmaes_batch_t* b) {
  if (!b) return fail(CMAES_EINVAL, "null batch");
  if (int rc = lockstep_generation(b->grp, b->inst)) return rc;
  // restart-on-finish with the same population size
  for (size_t k = 0; k < b->inst.size(); ++k) {
    cmaes* h = b->inst[k];
    uint32_t stop = 0;
    if (int rc = read_stop_best(h, &stop, nullptr, !b->grp.synced)) return rc;
    if (stop) {
      if (int rc = restart_same_lambda(h)) return rc;
      b->restarts[k] += 1;
    }
  }
  return CMAES_OK;
}

int cmaes_batch_state(const cmaes_batch_t* b, int k, cmaes_state_t* out) {
  if (int rc = batch_check(b, k)) return rc;
  return cmaes_state(b->inst[k], out);
}

int cmaes_batch_best(const cmaes_batch_t* b, double* f_best, int* k_best) {
  if (!b) return fail(CMAES_EINVAL, "null batch");
  double best = HUGE_VAL;
  int arg = -1;
  for (size_t k = 0; k < b->inst.size(); ++k) {
    double fb = HUGE_VAL;
    if (int rc = read_stop_best(b->inst[k], nullptr, &fb)) return rc;
    if (fb < best) {
      best = fb;
      arg = static_cast<int>(k);
    }
  }
  if (f_best) *f_best = best;
  if (k_best) *k_best = arg;
  return CMAES_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// K-Replicated strategy (Sec. 3.2.2, Alg. 3) on one GPU.  The resources that
// the paper splits into communicator halves are here the evaluation slots of
// one lockstep generation: k_max descents with lambda_start each start at
// once (the leaves of a binary tree); whenever both children of a tree node
// have finished, the node's descent starts with twice their population size
// (it takes over the left child's handle through an IPOP restart, the right
// child's handle is released), so the number of evaluations per lockstep
// generation stays k_max * lambda_start while descents run, until the root
// descent (lambda_start * k_max) finishes.  Every leaf has its own seed; a
// parent continues its left child's counter-based stream at the next restart
// index.

struct cmaes_krep {
  int n = 0, lam0 = 0, k_max = 1, levels = 0;
  cmaes_options_t opt{};
  bool have_opt = false;
  int obj_kind = CMAES_OBJ_NONE;
  std::vector<double> R, xstar;
  bool have_R = false, have_xstar = false;
  // node (level l, index j) is slot (2^(levels-l) - 1) + j of the arrays below
  std::vector<cmaes*> handle;      // running or finished-but-unmerged descent, else null
  std::vector<uint8_t> finished;   // descent of the node has finished
  std::vector<int32_t> gens;       // generations run by the node's descent
  int64_t released_evals = 0;      // evaluations of released handles
  double released_best = HUGE_VAL; // best f of released handles
  int64_t lockstep_gens = 0;
  bool done = false;
  LockstepGroup grp;
};

namespace {

int krep_slot(const cmaes_krep* r, int level, int j) { return ((1 << (r->levels - level)) - 1) + j; }

int krep_apply(cmaes_krep* r, cmaes* h) {
  if (r->have_opt) {
    cmaes_options_t o = r->opt;
    o.stream = nullptr;  // every descent on its own stream
    o.k_max = std::max(o.k_max, r->k_max);
    if (int rc = cmaes_set_options(h, &o)) return rc;
  } else {
    cmaes_options_t o;
    cmaes_get_options(h, &o);
    o.k_max = std::max(o.k_max, r->k_max);
    if (int rc = cmaes_set_options(h, &o)) return rc;
  }
  if (r->obj_kind != CMAES_OBJ_NONE)
    return cmaes_set_objective(h, r->obj_kind, r->have_R ? r->R.data() : nullptr,
                               r->have_xstar ? r->xstar.data() : nullptr);
  return 0;
}

}  // namespace

extern "C" {

cmaes_krep_t* cmaes_krep_create(int n, int lambda_start, int k_max, double sigma0, uint64_t seed) {
  if (n < 1 || k_max < 1 || k_max > 1024 || (k_max & (k_max - 1)) != 0) {
    set_error("cmaes_krep_create: n >= 1 and k_max a power of two in [1, 1024]");
    return nullptr;
  }
  cmaes_krep* r = new (std::nothrow) cmaes_krep();
  if (!r) {
    set_error("host allocation failed");
    return nullptr;
  }
  if (group_init(r->grp)) {
    const std::string why = g_err;
    cmaes_krep_destroy(r);
    set_error(why);
    return nullptr;
  }
  r->n = n;
  r->k_max = k_max;
  while ((1 << r->levels) < k_max) ++r->levels;
  const int nodes = 2 * k_max - 1;
  r->handle.assign(nodes, nullptr);
  r->finished.assign(nodes, 0);
  r->gens.assign(nodes, 0);
  for (int j = 0; j < k_max; ++j) {
    // distinct leaf seeds: the run's seed mixed with the leaf index
    const uint64_t s = seed * 0x9E3779B97F4A7C15ull + static_cast<uint64_t>(j) * 0xBF58476D1CE4E5B9ull + 1;
    cmaes* h = cmaes_create(n, lambda_start, sigma0, s);
    if (!h) {
      const std::string why = g_err;
      cmaes_krep_destroy(r);
      set_error("leaf " + std::to_string(j) + ": " + why);
      return nullptr;
    }
    r->handle[krep_slot(r, 0, j)] = h;
    r->lam0 = h->lam;
    if (krep_apply(r, h)) {
      const std::string why = g_err;
      cmaes_krep_destroy(r);
      set_error("leaf " + std::to_string(j) + ": " + why);
      return nullptr;
    }
  }
  return r;
}

void cmaes_krep_destroy(cmaes_krep_t* r) {
  if (!r) return;
  group_destroy(r->grp);
  for (cmaes* h : r->handle) cmaes_destroy(h);
  delete r;
}

int cmaes_krep_set_options(cmaes_krep_t* r, const cmaes_options_t* o) {
  if (!r || !o) return fail(CMAES_EINVAL, "null argument");
  r->opt = *o;
  r->have_opt = true;
  for (cmaes* h : r->handle)
    if (h)
      if (int rc = krep_apply(r, h)) return rc;
  return CMAES_OK;
}

int cmaes_krep_set_objective(cmaes_krep_t* r, int kind, const double* R, const double* xstar) {
  if (!r) return fail(CMAES_EINVAL, "null argument");
  if (kind < CMAES_OBJ_NONE || kind > CMAES_OBJ_RASTRIGIN) return fail(CMAES_EINVAL, "unknown objective");
  const size_t n = static_cast<size_t>(r->n);
  r->obj_kind = kind;
  r->have_R = R != nullptr;
  r->have_xstar = xstar != nullptr;
  r->R.assign(R ? R : R, R ? R + n * n : R);
  r->xstar.assign(xstar ? xstar : xstar, xstar ? xstar + n : xstar);
  for (cmaes* h : r->handle)
    if (h)
      if (int rc = cmaes_set_objective(h, kind, R, xstar)) return rc;
  return CMAES_OK;
}

int cmaes_krep_generation(cmaes_krep_t* r) {
  if (!r) return fail(CMAES_EINVAL, "null argument");
  if (r->done) return CMAES_OK;
  std::vector<cmaes*> run;
  std::vector<int> slot;
  for (int l = 0; l <= r->levels; ++l)
    for (int j = 0; j < (r->k_max >> l); ++j) {
      const int s = krep_slot(r, l, j);
      if (r->handle[s] && !r->finished[s]) {
        run.push_back(r->handle[s]);
        slot.push_back(s);
      }
    }
  if (int rc = lockstep_generation(r->grp, run)) return rc;
  r->lockstep_gens += 1;
  double best = r->released_best;
  // the members' streams are idle after a synchronised lockstep generation,
  // and the other descents' streams were left idle by their last call
  const bool sync = !r->grp.synced;
  for (size_t i = 0; i < run.size(); ++i) {
    uint32_t stop = 0;
    if (int rc = read_stop_best(run[i], &stop, nullptr, sync)) return rc;
    r->gens[slot[i]] += 1;
    if (stop) r->finished[slot[i]] = 1;
  }
  for (cmaes* h : r->handle)
    if (h) {
      double fb = HUGE_VAL;
      if (int rc = read_stop_best(h, nullptr, &fb, sync)) return rc;
      best = std::min(best, fb);
    }
  // merge finished sibling pairs into their parent (Alg. 3: the control flows
  // back to the parent communicator once both halves are done)
  for (int l = 1; l <= r->levels; ++l)
    for (int j = 0; j < (r->k_max >> l); ++j) {
      const int p = krep_slot(r, l, j), a = krep_slot(r, l - 1, 2 * j), b = krep_slot(r, l - 1, 2 * j + 1);
      if (r->handle[p] || r->finished[p] || !r->finished[a] || !r->finished[b]) continue;
      cmaes* hb = r->handle[b];
      if (hb) {
        double fb = HUGE_VAL;
        if (int rc = read_stop_best(hb, nullptr, &fb, sync)) return rc;
        r->released_best = std::min(r->released_best, fb);
        r->released_evals += hb->total_evals;
        r->handle[b] = nullptr;
        cmaes_destroy(hb);
      }
      cmaes* ha = r->handle[a];
      r->handle[a] = nullptr;
      r->handle[p] = ha;
      if (int rc = cmaes_restart_ipop(ha)) return rc;
    }
  const int root = krep_slot(r, r->levels, 0);
  const bool target = r->have_opt ? best < r->opt.f_target : best < 1e-8;
  r->done = r->finished[root] || target;
  return CMAES_OK;
}

int cmaes_krep_status(const cmaes_krep_t* r, cmaes_krep_status_t* out) {
  if (!r || !out) return fail(CMAES_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  double best = r->released_best;
  int64_t evals = r->released_evals;
  int32_t lmax = 0;
  for (int l = 0; l <= r->levels; ++l)
    for (int j = 0; j < (r->k_max >> l); ++j) {
      const int s = krep_slot(r, l, j);
      if (r->finished[s]) out->finished += 1;
      cmaes* h = r->handle[s];
      if (!h) continue;
      if (!r->finished[s]) {
        out->running += 1;
        lmax = std::max(lmax, h->lam);
      }
      double fb = HUGE_VAL;
      // after a synchronised lockstep generation every descent's stream is idle
      if (int rc = read_stop_best(h, nullptr, &fb, !r->grp.synced)) return rc;
      best = std::min(best, fb);
      evals += h->total_evals;
    }
  out->lambda_max_running = lmax;
  out->done = r->done ? 1 : 0;
  out->lockstep_generations = r->lockstep_gens;
  out->total_evals = evals;
  out->f_best = best;
  return CMAES_OK;
}

int cmaes_krep_run(cmaes_krep_t* r, int64_t max_lockstep_generations) {
  if (!r) return fail(CMAES_EINVAL, "null argument");
  for (int64_t g = 0; !r->done && g < max_lockstep_generations; ++g)
    if (int rc = cmaes_krep_generation(r)) return rc;
  return CMAES_OK;
}

}  // extern "C"
