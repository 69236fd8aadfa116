// Ranking, recombination and the float64 vector updates of one generation
// (Alg. 1 'update' line, Sec. 2.1), plus the stopping tests (Sec. 2.2).
//
// Readings shared with the oracle (no formula is printed in the paper):
// tutorial default rates, positive weights w_1..w_mu summing to one, the
// cumulative step-size path p_sigma built from C^{-1/2} y_w = B z_w, the
// h_sigma stall of p_c, sigma <- sigma exp((cs/ds)(||p_sigma||/chi_n - 1)).
// All reductions use a fixed order (no floating-point atomics), so a run is
// bitwise reproducible.
#include "internal.h"

namespace cmx {

namespace {

__device__ __forceinline__ double rank_key(double v) { return v != v ? __builtin_inf() : v; }

// ---- ranking by chunk sort and merge: the keys (f, index), NaN counted as
// +inf, are cut into chunks of kSortChunk; each chunk is sorted by a bitonic
// network in LDS (k_chunk_sort); the rank of a key is its position in its own
// chunk plus, for every other chunk, the number of that chunk's keys below
// it, found by binary search (k_merge_count, chunks taken kMergeGroup at a
// time from LDS, one partial count per group); k_merge_scatter sums the
// counts and writes order[rank] = index.  The keys are distinct, so the ranks
// form the stable ascending permutation exactly; the counts are integers.
constexpr int kSortChunk = 256, kMergeGroup = 8;

__device__ __forceinline__ bool key_less(double ka, int ia, double kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// the sorted chunks: keys in skey (double), indices in sidx; padding entries
// (+inf, INT_MAX) sort after every real key
__device__ __forceinline__ void chunk_sort_body(int c, const double* __restrict__ f, int lam,
                                                double* __restrict__ skey, int* __restrict__ sidx) {
  __shared__ double k[kSortChunk];
  __shared__ int ix[kSortChunk];
  const int t = threadIdx.x, i = c * kSortChunk + t;
  k[t] = i < lam ? rank_key(f[i]) : __builtin_inf();
  ix[t] = i < lam ? i : 0x7fffffff;
  for (int size = 2; size <= kSortChunk; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      const int u = t ^ stride;
      if (u > t) {
        const bool up = (t & size) == 0;
        const double ka = k[t], kb = k[u];
        const int ia = ix[t], ib = ix[u];
        if (key_less(kb, ib, ka, ia) == up) {
          k[t] = kb;
          ix[t] = ib;
          k[u] = ka;
          ix[u] = ia;
        }
      }
    }
  __syncthreads();
  skey[i] = k[t];
  sidx[i] = ix[t];
}

__global__ void __launch_bounds__(256) k_chunk_sort(const double* __restrict__ f, int lam, double* __restrict__ skey,
                                                    int* __restrict__ sidx) {
  chunk_sort_body(blockIdx.x, f, lam, skey, sidx);
}

// workgroup (c, g): the keys of chunk c counted against chunks
// [g kMergeGroup, (g + 1) kMergeGroup) other than c
__device__ __forceinline__ void merge_count_body(int c, int g, int nchunks, const double* __restrict__ skey,
                                                 const int* __restrict__ sidx, int lam, int32_t* __restrict__ part) {
  __shared__ double ok[kSortChunk];
  __shared__ int oi[kSortChunk];
  const int t = threadIdx.x;
  const double kt = skey[c * kSortChunk + t];
  const int it = sidx[c * kSortChunk + t];
  int cnt = 0;
  const int c1 = min(nchunks, (g + 1) * kMergeGroup);
  for (int o = g * kMergeGroup; o < c1; ++o) {
    if (o == c) continue;  // uniform over the workgroup
    __syncthreads();
    ok[t] = skey[o * kSortChunk + t];
    oi[t] = sidx[o * kSortChunk + t];
    __syncthreads();
    int lo = 0, hi = kSortChunk;  // the first entry not below (kt, it)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (key_less(ok[mid], oi[mid], kt, it))
        lo = mid + 1;
      else
        hi = mid;
    }
    cnt += lo;
  }
  if (it < lam) part[static_cast<int64_t>(g) * lam + it] = cnt;
}

__global__ void __launch_bounds__(256) k_merge_count(int nchunks, const double* __restrict__ skey,
                                                     const int* __restrict__ sidx, int lam,
                                                     int32_t* __restrict__ part) {
  merge_count_body(blockIdx.x, blockIdx.y, nchunks, skey, sidx, lam, part);
}

__device__ __forceinline__ void merge_scatter_body(int c, int ngroups, const int* __restrict__ sidx, int lam,
                                                   const int32_t* __restrict__ part, int32_t* __restrict__ order) {
  const int t = threadIdx.x;
  const int i = sidx[c * kSortChunk + t];
  if (i >= lam) return;
  int rank = t;
  for (int g = 0; g < ngroups; ++g) rank += part[static_cast<int64_t>(g) * lam + i];
  order[rank] = i;
}

__global__ void __launch_bounds__(256) k_merge_scatter(int ngroups, const int* __restrict__ sidx, int lam,
                                                       const int32_t* __restrict__ part, int32_t* __restrict__ order) {
  merge_scatter_body(blockIdx.x, ngroups, sidx, lam, part, order);
}

// y_w = sum_{r<mu} w_r y_{order[r]}, z_w likewise (float64 accumulation), and
// Yhat[:, r] = sqrt(w_r) y_{order[r]} for the rank-mu SYRK.  Grid: rows x
// chunks of 64 ranks; each chunk writes its own partial sums.
template <typename T>
__device__ __forceinline__ void recombine_body(int bx, int by, int n, int mu, const T* __restrict__ Y,
                                               const T* __restrict__ Z, int ld, const int32_t* __restrict__ order,
                                               const double* __restrict__ w, const double* __restrict__ sqrtw,
                                               T* __restrict__ Ysel, int ldsel, double* __restrict__ part_yw,
                                               double* __restrict__ part_zw) {
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r0 = by * 64, r1 = min(mu, r0 + 64);
  double ay = 0.0, az = 0.0;
  // unrolled so that many loads are in flight; the sums keep rank order
#pragma unroll 16
  for (int r = r0; r < r1; ++r) {
    const int64_t c = static_cast<int64_t>(order[r]) * ld;
    const T y = Y[c + i];
    const T z = Z[c + i];
    ay += w[r] * static_cast<double>(y);
    az += w[r] * static_cast<double>(z);
    Ysel[static_cast<int64_t>(r) * ldsel + i] = static_cast<T>(sqrtw[r] * static_cast<double>(y));
  }
  part_yw[static_cast<int64_t>(by) * n + i] = ay;
  part_zw[static_cast<int64_t>(by) * n + i] = az;
}

template <typename T>
__global__ void __launch_bounds__(256) k_recombine(int n, int mu, const T* __restrict__ Y,
                                                   const T* __restrict__ Z, int ld,
                                                   const int32_t* __restrict__ order,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ sqrtw, T* __restrict__ Ysel,
                                                   int ldsel, double* __restrict__ part_yw,
                                                   double* __restrict__ part_zw) {
  recombine_body<T>(blockIdx.x, blockIdx.y, n, mu, Y, Z, ld, order, w, sqrtw, Ysel, ldsel, part_yw, part_zw);
}

__device__ __forceinline__ void reduce_yz_body(int bx, int n, int nchunks, const double* __restrict__ py,
                                               const double* __restrict__ pz, double* __restrict__ yw,
                                               double* __restrict__ zw) {
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0, b = 0.0;
#pragma unroll 16
  for (int c = 0; c < nchunks; ++c) {
    a += py[static_cast<int64_t>(c) * n + i];
    b += pz[static_cast<int64_t>(c) * n + i];
  }
  yw[i] = a;
  zw[i] = b;
}

__global__ void k_reduce_yz(int n, int nchunks, const double* __restrict__ py, const double* __restrict__ pz,
                            double* __restrict__ yw, double* __restrict__ zw) {
  reduce_yz_body(blockIdx.x, n, nchunks, py, pz, yw, zw);
}

// part[c][i] = sum_{j in chunk c} B[i + j ld] x[j]
__device__ __forceinline__ void matvec_body(int bx, int by, int n, const double* __restrict__ B, int ldb,
                                            const double* __restrict__ x, double* __restrict__ part) {
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j0 = by * 64, j1 = min(n, j0 + 64);
  double s = 0.0;
#pragma unroll 16
  for (int j = j0; j < j1; ++j) s += B[static_cast<int64_t>(j) * ldb + i] * x[j];
  part[static_cast<int64_t>(by) * n + i] = s;
}

__global__ void __launch_bounds__(256) k_matvec(int n, const double* __restrict__ B, int ldb,
                                                const double* __restrict__ x, double* __restrict__ part) {
  matvec_body(blockIdx.x, blockIdx.y, n, B, ldb, x, part);
}

template <int NT>
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// p_sigma, h_sigma, p_c, m, sigma and the covariance coefficient a.
__device__ __forceinline__ void vec_update_body(const KParams& kp, int nchunks, const double* __restrict__ part_bz,
                                                const double* __restrict__ yw, double* __restrict__ m,
                                                double* __restrict__ ps, double* __restrict__ pc,
                                                DevScalars* __restrict__ sc) {
  __shared__ double red[1024];
  const int n = kp.n;
  const double sigma = sc->sigma;
  const int64_t g = sc->gen;
  const double fps = sqrt(kp.cs * (2.0 - kp.cs) * kp.mueff);
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    double bz = 0.0;
#pragma unroll 16
    for (int c = 0; c < nchunks; ++c) bz += part_bz[static_cast<int64_t>(c) * n + i];
    const double v = (1.0 - kp.cs) * ps[i] + fps * bz;
    ps[i] = v;
    acc += v * v;
  }
  const double nps = sqrt(block_sum<1024>(acc, red));
  const double denom = sqrt(1.0 - pow(1.0 - kp.cs, 2.0 * static_cast<double>(g + 1)));
  const double hsig = (nps / denom < (1.4 + 2.0 / (n + 1.0)) * kp.chin) ? 1.0 : 0.0;
  const double fpc = hsig * sqrt(kp.cc * (2.0 - kp.cc) * kp.mueff);
  for (int i = threadIdx.x; i < n; i += 1024) {
    pc[i] = (1.0 - kp.cc) * pc[i] + fpc * yw[i];
    m[i] = m[i] + sigma * yw[i];
  }
  if (threadIdx.x == 0) {
    sc->ps_norm = nps;
    sc->hsig = hsig;
    sc->c_coef = 1.0 - kp.c1 - kp.cmu * kp.sumw + (1.0 - hsig) * kp.c1 * kp.cc * (2.0 - kp.cc);
    sc->sigma = sigma * exp((kp.cs / kp.ds) * (nps / kp.chin - 1.0));
    sc->gen = g + 1;
    sc->evals += kp.lam;
  }
}

__global__ void __launch_bounds__(1024) k_vec_update(KParams kp, int nchunks, const double* __restrict__ part_bz,
                                                     const double* __restrict__ yw, double* __restrict__ m,
                                                     double* __restrict__ ps, double* __restrict__ pc,
                                                     DevScalars* __restrict__ sc) {
  vec_update_body(kp, nchunks, part_bz, yw, m, ps, pc, sc);
}

// Best-so-far point and the f-history ring; runs before m and sigma move.
template <typename T>
__device__ __forceinline__ void best_body(int n, int lam, const double* __restrict__ f,
                                          const int32_t* __restrict__ order, const T* __restrict__ Y, int ldy,
                                          const double* __restrict__ m, double* __restrict__ x_best,
                                          double* __restrict__ hist, int hist_len, DevScalars* __restrict__ sc) {
  const int i0 = order[0];
  const double f0 = rank_key(f[i0]);
  const double flast = rank_key(f[order[lam - 1]]);
  const bool better = f0 < sc->f_best;
  if (better) {
    const double sigma = sc->sigma;
    const T* y = Y + static_cast<int64_t>(i0) * ldy;
    for (int i = threadIdx.x; i < n; i += blockDim.x) x_best[i] = m[i] + sigma * static_cast<double>(y[i]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    hist[sc->hist_count % hist_len] = f0;
    sc->hist_count += 1;
    sc->f_gen_min = f0;
    sc->f_gen_max = flast;
    if (better) sc->f_best = f0;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_best(int n, int lam, const double* __restrict__ f,
                                              const int32_t* __restrict__ order, const T* __restrict__ Y,
                                              int ldy, const double* __restrict__ m, double* __restrict__ x_best,
                                              double* __restrict__ hist, int hist_len,
                                              DevScalars* __restrict__ sc) {
  best_body<T>(n, lam, f, order, Y, ldy, m, x_best, hist, hist_len, sc);
}

__device__ __forceinline__ int block_or(int v, int* red) {
  __syncthreads();
  if (threadIdx.x == 0) *red = 0;
  __syncthreads();
  if (v) atomicOr(red, v);
  __syncthreads();
  return *red;
}

__device__ __forceinline__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Stopping tests evaluated after the update (reading of Sec. 2.2; thresholds
// of the original IPOP-CMA-ES paper).
__device__ __forceinline__ void stop_body(const KParams& kp, const StopParams& sp, const double* __restrict__ m,
                                          const double* __restrict__ C, int ldc, const double* __restrict__ B,
                                          int ldb, const double* __restrict__ D, const double* __restrict__ pc,
                                          const double* __restrict__ hist, DevScalars* __restrict__ sc,
                                          uint32_t* __restrict__ hstop) {
  __shared__ double red[256];
  __shared__ int ired;
  const int n = kp.n;
  const double sigma = sc->sigma;
  const int64_t g = sc->gen;
  const int ax = static_cast<int>(g % n);
  double maxsd = 0.0, maxpc = 0.0, dmax = 0.0, dmin_neg = -__builtin_inf();
  int axis_moves = 0, coord_stuck = 0, nonfinite = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double cii = C[static_cast<int64_t>(i) * ldc + i];
    const double sd = sqrt(cii);
    maxsd = fmax(maxsd, sd);
    maxpc = fmax(maxpc, fabs(pc[i]));
    dmax = fmax(dmax, D[i]);
    dmin_neg = fmax(dmin_neg, -D[i]);
    const double mi = m[i];
    if (mi + 0.1 * sigma * D[ax] * B[static_cast<int64_t>(ax) * ldb + i] != mi) axis_moves = 1;
    if (mi + 0.2 * sigma * sd == mi) coord_stuck = 1;
    if (!isfinite(mi) || !isfinite(cii) || !isfinite(pc[i]) || !isfinite(D[i])) nonfinite = 1;
  }
  maxsd = block_max(maxsd, red);
  maxpc = block_max(maxpc, red);
  dmax = block_max(dmax, red);
  const double dmin = -block_max(dmin_neg, red);
  axis_moves = block_or(axis_moves, &ired);
  coord_stuck = block_or(coord_stuck, &ired);
  nonfinite = block_or(nonfinite, &ired);
  if (threadIdx.x != 0) return;
  uint32_t bits = 0;
  const int cnt = sc->hist_count;
  if (cnt >= sp.hist_len) {
    double hmin = __builtin_inf(), hmax = -__builtin_inf();
    for (int q = 0; q < sp.hist_len; ++q) {
      const double h = hist[(cnt - 1 - q) % sp.hist_len];
      hmin = fmin(hmin, h);
      hmax = fmax(hmax, h);
    }
    if (hmax - hmin < sp.tol_hist_fun) bits |= 1u << 0;
    if (fmax(hmax, sc->f_gen_max) - fmin(hmin, sc->f_gen_min) < sp.tol_fun) bits |= 1u << 1;
  }
  if (sigma * maxsd < sp.tolx && sigma * maxpc < sp.tolx) bits |= 1u << 2;
  if (!axis_moves) bits |= 1u << 3;
  if (coord_stuck) bits |= 1u << 4;
  if (!sc->eig_ok || !(dmin > 0.0) || (dmax / dmin) * (dmax / dmin) > sp.max_condition) bits |= 1u << 5;
  if (sc->f_best < sp.f_target) bits |= 1u << 6;
  if (sp.max_gens > 0 && g >= sp.max_gens) bits |= 1u << 7;
  if (sp.max_evals > 0 && sc->evals >= sp.max_evals) bits |= 1u << 8;
  if (nonfinite || !isfinite(sigma)) bits |= 1u << 9;
  sc->stop = bits;
  // the host's copy of the bits and of f_best (pinned, mapped host memory:
  // the bits at hstop[0], f_best at hstop[2..3]): system-scope stores, read
  // by the host after the end of this kernel
  if (hstop) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(hstop + 2),
                       static_cast<unsigned long long>(__double_as_longlong(sc->f_best)), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(hstop, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ void __launch_bounds__(256) k_stop(KParams kp, StopParams sp, const double* __restrict__ m,
                                              const double* __restrict__ C, int ldc,
                                              const double* __restrict__ B, int ldb,
                                              const double* __restrict__ D, const double* __restrict__ pc,
                                              const double* __restrict__ hist, DevScalars* __restrict__ sc,
                                              uint32_t* __restrict__ hstop) {
  stop_body(kp, sp, m, C, ldc, B, ldb, D, pc, hist, sc, hstop);
}

// u = m - x* (x* may be null = origin)
__device__ __forceinline__ void sub_body(int bx, int n, const double* __restrict__ m, const double* __restrict__ xs,
                                         double* __restrict__ u) {
  const int i = bx * blockDim.x + threadIdx.x;
  if (i < n) u[i] = m[i] - (xs ? xs[i] : 0.0);
}

__global__ void k_sub(int n, const double* __restrict__ m, const double* __restrict__ xs, double* __restrict__ u) {
  sub_body(blockIdx.x, n, m, xs, u);
}

__device__ __forceinline__ void reduce_vec_body(int bx, int n, int nchunks, const double* __restrict__ part,
                                                double* __restrict__ out) {
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
#pragma unroll 16
  for (int c = 0; c < nchunks; ++c) a += part[static_cast<int64_t>(c) * n + i];
  out[i] = a;
}

__global__ void k_reduce_vec(int n, int nchunks, const double* __restrict__ part, double* __restrict__ out) {
  reduce_vec_body(blockIdx.x, n, nchunks, part, out);
}

__global__ void k_set_identity(double* A, int n, int ld) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * ld) return;
  const int col = static_cast<int>(idx / ld), row = static_cast<int>(idx % ld);
  A[idx] = (row == col) ? 1.0 : 0.0;
}

template <typename T>
__global__ void k_convert(const double* __restrict__ s, int lds, T* __restrict__ d, int ldd, int rows,
                          int cols) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(rows) * cols) return;
  const int c = static_cast<int>(idx / rows), r = static_cast<int>(idx % rows);
  d[static_cast<int64_t>(c) * ldd + r] = static_cast<T>(s[static_cast<int64_t>(c) * lds + r]);
}

}  // namespace


// the rank work area (int32 elements): sorted keys (double, 2 words each),
// their indices, then the per-group counts
struct RankWork {
  double* skey;
  int* sidx;
  int32_t* part;
  int nchunks, ngroups;
};
__host__ __device__ inline RankWork rank_work_of(int32_t* work, int lam) {
  RankWork w;
  w.nchunks = (lam + kSortChunk - 1) / kSortChunk;
  w.ngroups = (w.nchunks + kMergeGroup - 1) / kMergeGroup;
  w.skey = reinterpret_cast<double*>(work);
  w.sidx = work + 2 * w.nchunks * kSortChunk;
  w.part = w.sidx + w.nchunks * kSortChunk;
  return w;
}

hipError_t launch_rank(hipStream_t st, const double* f, int lam, int32_t* order, int32_t* work) {
  const RankWork w = rank_work_of(work, lam);
  k_chunk_sort<<<w.nchunks, 256, 0, st>>>(f, lam, w.skey, w.sidx);
  if (w.nchunks > 1) k_merge_count<<<dim3(w.nchunks, w.ngroups), 256, 0, st>>>(w.nchunks, w.skey, w.sidx, lam, w.part);
  k_merge_scatter<<<w.nchunks, 256, 0, st>>>(w.nchunks > 1 ? w.ngroups : 0, w.sidx, lam, w.part, order);
  return hipGetLastError();
}

size_t rank_work_elems(int lam) {
  const size_t nchunks = ceil_div(lam, kSortChunk), ngroups = ceil_div(static_cast<int>(nchunks), kMergeGroup);
  return 3 * nchunks * kSortChunk + ngroups * static_cast<size_t>(lam) + 2;
}

hipError_t launch_recombine(hipStream_t st, bool fp64, int n, int lam, int mu, const void* Y, const void* Z,
                            int ld, const int32_t* order, const double* w, const double* sqrtw, void* Ysel,
                            int ldsel, double* part_yw, double* part_zw, int* nchunks) {
  (void)lam;
  *nchunks = ceil_div(mu, 64);
  dim3 grid(ceil_div(n, 256), *nchunks);
  if (fp64)
    k_recombine<double><<<grid, 256, 0, st>>>(n, mu, static_cast<const double*>(Y),
                                              static_cast<const double*>(Z), ld, order, w, sqrtw,
                                              static_cast<double*>(Ysel), ldsel, part_yw, part_zw);
  else
    k_recombine<float><<<grid, 256, 0, st>>>(n, mu, static_cast<const float*>(Y), static_cast<const float*>(Z),
                                             ld, order, w, sqrtw, static_cast<float*>(Ysel), ldsel, part_yw,
                                             part_zw);
  return hipGetLastError();
}

hipError_t launch_reduce_yz(hipStream_t st, int n, int nchunks, const double* part_yw, const double* part_zw,
                            double* yw, double* zw) {
  k_reduce_yz<<<ceil_div(n, 256), 256, 0, st>>>(n, nchunks, part_yw, part_zw, yw, zw);
  return hipGetLastError();
}

hipError_t launch_matvec(hipStream_t st, int n, const double* B, int ldb, const double* x, double* part,
                         int* nchunks) {
  *nchunks = ceil_div(n, 64);
  dim3 grid(ceil_div(n, 256), *nchunks);
  k_matvec<<<grid, 256, 0, st>>>(n, B, ldb, x, part);
  return hipGetLastError();
}

hipError_t launch_vec_update(hipStream_t st, const KParams& kp, int nchunks, const double* part_bz,
                             const double* yw, double* m, double* ps, double* pc, DevScalars* sc) {
  k_vec_update<<<1, 1024, 0, st>>>(kp, nchunks, part_bz, yw, m, ps, pc, sc);
  return hipGetLastError();
}

hipError_t launch_best(hipStream_t st, bool fp64, int n, int lam, const double* f, const int32_t* order,
                       const void* Y, int ldy, const double* m, double* x_best, double* hist, int hist_len,
                       DevScalars* sc) {
  if (fp64)
    k_best<double><<<1, 256, 0, st>>>(n, lam, f, order, static_cast<const double*>(Y), ldy, m, x_best, hist,
                                      hist_len, sc);
  else
    k_best<float><<<1, 256, 0, st>>>(n, lam, f, order, static_cast<const float*>(Y), ldy, m, x_best, hist,
                                     hist_len, sc);
  return hipGetLastError();
}

hipError_t launch_stop(hipStream_t st, const KParams& kp, const StopParams& sp, const double* m,
                       const double* C, int ldc, const double* B, int ldb, const double* D,
                       const double* pc, const double* hist, DevScalars* sc, uint32_t* hstop) {
  k_stop<<<1, 256, 0, st>>>(kp, sp, m, C, ldc, B, ldb, D, pc, hist, sc, hstop);
  return hipGetLastError();
}

hipError_t launch_shift(hipStream_t st, int n, const double* R, int ldr, const double* m, const double* xstar,
                        double* u, double* part, double* d) {
  k_sub<<<ceil_div(n, 256), 256, 0, st>>>(n, m, xstar, R ? u : d);
  if (R) {
    const int nch = ceil_div(n, 64);
    dim3 grid(ceil_div(n, 256), nch);
    k_matvec<<<grid, 256, 0, st>>>(n, R, ldr, u, part);
    k_reduce_vec<<<ceil_div(n, 256), 256, 0, st>>>(n, nch, part, d);
  }
  return hipGetLastError();
}

// B <- (3 B - B (B^T B)) / 2 from T = B (B^T B): one Newton-Schulz step
// towards the orthogonal polar factor of B (rows < n only)
__device__ __forceinline__ void polar_body(int bx, int n, double* __restrict__ B, int ldb, const double* __restrict__ T,
                                           int ldt) {
  const int64_t idx = static_cast<int64_t>(bx) * blockDim.x + threadIdx.x;
  const int64_t total = static_cast<int64_t>(n) * n;
  if (idx >= total) return;
  const int col = static_cast<int>(idx / n), row = static_cast<int>(idx % n);
  double& b = B[static_cast<int64_t>(col) * ldb + row];
  b = 1.5 * b - 0.5 * T[static_cast<int64_t>(col) * ldt + row];
}

__global__ void k_polar_step(int n, double* __restrict__ B, int ldb, const double* __restrict__ T, int ldt) {
  polar_body(blockIdx.x, n, B, ldb, T, ldt);
}

// ---- variants

// active covariance update: one workgroup per rank r; ranks beyond mu get the
// negative weight scaled by n / ||C^{-1/2} y||^2 = n / ||z||^2 (y = B D z with
// orthonormal B), the norm summed in float64 in a fixed order
template <typename T>
__global__ void __launch_bounds__(256) k_active_cols(int n, int mu, const T* __restrict__ Y, const T* __restrict__ Z,
                                                     int ld, const int32_t* __restrict__ order,
                                                     const double* __restrict__ w_all, T* __restrict__ Ysel,
                                                     T* __restrict__ Ysig, int ldsel) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  T* ys = Ysel + static_cast<int64_t>(r) * ldsel;
  T* yg = Ysig + static_cast<int64_t>(r) * ldsel;
  if (r < mu) {  // the positive columns, as the recombination wrote them
    for (int i = threadIdx.x; i < n; i += 256) yg[i] = ys[i];
    return;
  }
  const int64_t c = static_cast<int64_t>(order[r]) * ld;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double z = static_cast<double>(Z[c + i]);
    acc += z * z;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double wr = w_all[r], z2 = red[0];
  const double sc = (wr < 0.0 && z2 > 0.0) ? sqrt(-wr * n / z2) : 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double v = sc * static_cast<double>(Y[c + i]);
    ys[i] = static_cast<T>(v);
    yg[i] = static_cast<T>(-v);
  }
}

// separable sampling: y = D z
template <typename T>
__global__ void __launch_bounds__(256) k_sep_sample(int n, int lam, const double* __restrict__ D,
                                                    const T* __restrict__ Z, int ldz, T* __restrict__ Y, int ldy) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * lam) return;
  const int k = static_cast<int>(idx / n), i = static_cast<int>(idx % n);
  Y[static_cast<int64_t>(k) * ldy + i] = static_cast<T>(D[i] * static_cast<double>(Z[static_cast<int64_t>(k) * ldz + i]));
}

// separable covariance update: the diagonal of the rank-one plus rank-mu update
template <typename T>
__global__ void __launch_bounds__(256) k_sep_cov(int n, int mu, const T* __restrict__ Y, int ldy,
                                                 const int32_t* __restrict__ order, const double* __restrict__ w,
                                                 const double* __restrict__ pc, double c1, double cmu,
                                                 double* __restrict__ C, int ldc, const DevScalars* __restrict__ sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int r = 0; r < mu; ++r) {
    const double y = static_cast<double>(Y[static_cast<int64_t>(order[r]) * ldy + i]);
    acc += w[r] * y * y;
  }
  double& cii = C[static_cast<int64_t>(i) * ldc + i];
  cii = sc->c_coef * cii + c1 * pc[i] * pc[i] + cmu * acc;
}

// separable "decomposition": D = sqrt(diag C), B D = diag(D); eig_ok when the
// diagonal is positive (a one-workgroup kernel)
template <typename T>
__global__ void __launch_bounds__(256) k_sep_eigen(int n, const double* __restrict__ C, int ldc,
                                                   double* __restrict__ D, T* __restrict__ BD, int ldbd,
                                                   DevScalars* __restrict__ sc) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    const double cii = C[static_cast<int64_t>(i) * ldc + i];
    if (!(cii > 0.0)) atomicOr(&bad, 1);
    const double d = sqrt(fmax(cii, 0.0));
    D[i] = d;
    BD[static_cast<int64_t>(i) * ldbd + i] = static_cast<T>(d);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sc->eig_ok = bad ? 0 : 1;
    sc->jac_sweeps = 0;
    sc->jac_corr = 0;
  }
}

// ---- the update steps of a grouped front (one launch per step for all
// descents; workgroup w of descent i is local block w - off[i], split into
// (bx, by) by the descent's own grid width)
__global__ void __launch_bounds__(256) kg_update256(int kind, const GFront* __restrict__ g, const int* __restrict__ off,
                                                    int count, GroupDueMask mask) {
  const int i = group_find(off, count, blockIdx.x);
  const GFront& e = g[i];
  const int w = blockIdx.x - off[i];
  const int gx = (e.n + 255) / 256;
  switch (kind) {
    case GF_SUB: sub_body(w, e.n, e.m, e.xstar, e.u); break;
    case GF_RMATVEC: matvec_body(w % gx, w / gx, e.n, e.Rd, e.ldn, e.u, e.part_bz); break;
    case GF_RVEC: reduce_vec_body(w, e.n, (e.n + 63) / 64, e.part_bz, e.d); break;
    case GF_RANK: {
      const RankWork rw = rank_work_of(e.rank_work, e.lam);
      chunk_sort_body(w, e.f, e.lam, rw.skey, rw.sidx);
      break;
    }
    case GF_MERGE: {
      const RankWork rw = rank_work_of(e.rank_work, e.lam);
      merge_count_body(w % rw.nchunks, w / rw.nchunks, rw.nchunks, rw.skey, rw.sidx, e.lam, rw.part);
      break;
    }
    case GF_SCATTER: {
      const RankWork rw = rank_work_of(e.rank_work, e.lam);
      merge_scatter_body(w, rw.nchunks > 1 ? rw.ngroups : 0, rw.sidx, e.lam, rw.part, e.order);
      break;
    }
    case GF_BEST: best_body<float>(e.n, e.lam, e.f, e.order, e.Y, e.ldn, e.m, e.x_best, e.hist, e.hist_len, e.sc); break;
    case GF_RECOMB:
      recombine_body<float>(w % gx, w / gx, e.n, e.mu, e.Y, e.Z, e.ldn, e.order, e.w, e.sqrtw, e.Ysel, e.ldn,
                            e.part_yw, e.part_zw);
      break;
    case GF_REDYZ: reduce_yz_body(w, e.n, (e.mu + 63) / 64, e.part_yw, e.part_zw, e.yw, e.zw); break;
    case GF_BMATVEC: matvec_body(w % gx, w / gx, e.n, e.B, e.ldn, e.zw, e.part_bz); break;
    case GF_POLAR:
      if (due_mask_bit(mask, i)) polar_body(w, e.n, e.B, e.ldn, e.T, e.ldn);
      break;
    case GF_STOP: stop_body(e.kp, e.sp, e.m, e.C, e.ldn, e.B, e.ldn, e.D, e.pc, e.hist, e.sc, e.hstop); break;
    default: break;
  }
}

__global__ void __launch_bounds__(1024) kg_vec_update(const GFront* __restrict__ g, const int* __restrict__ off,
                                                      int count) {
  const int i = group_find(off, count, blockIdx.x);
  const GFront& e = g[i];
  vec_update_body(e.kp, (e.n + 63) / 64, e.part_bz, e.yw, e.m, e.ps, e.pc, e.sc);
}

hipError_t launch_group_update(hipStream_t st, int kind, const GFront* g, const int* off, int count, int wgs,
                               const GroupDueMask* mask) {
  if (wgs == 0) return hipSuccess;
  if (kind == GF_VECUPD) {
    kg_vec_update<<<wgs, 1024, 0, st>>>(g, off, count);
  } else {
    GroupDueMask m{};
    if (mask) m = *mask;
    kg_update256<<<wgs, 256, 0, st>>>(kind, g, off, count, m);
  }
  return hipGetLastError();
}

int rank_chunks(int lam) { return ceil_div(lam, kSortChunk); }
int rank_merge_wgs(int lam) {
  const int nch = ceil_div(lam, kSortChunk);
  return nch > 1 ? nch * ceil_div(nch, kMergeGroup) : 0;
}

hipError_t launch_active_cols(hipStream_t st, bool fp64, int n, int lam, int mu, const void* Y, const void* Z, int ld,
                              const int32_t* order, const double* w_all, void* Ysel, void* Ysig, int ldsel) {
  if (fp64)
    k_active_cols<double><<<lam, 256, 0, st>>>(n, mu, static_cast<const double*>(Y), static_cast<const double*>(Z), ld,
                                               order, w_all, static_cast<double*>(Ysel), static_cast<double*>(Ysig),
                                               ldsel);
  else
    k_active_cols<float><<<lam, 256, 0, st>>>(n, mu, static_cast<const float*>(Y), static_cast<const float*>(Z), ld,
                                              order, w_all, static_cast<float*>(Ysel), static_cast<float*>(Ysig),
                                              ldsel);
  return hipGetLastError();
}

hipError_t launch_sep_sample(hipStream_t st, bool fp64, int n, int lam, const double* D, const void* Z, int ldz,
                             void* Y, int ldy) {
  const int64_t total = static_cast<int64_t>(n) * lam;
  const int blocks = static_cast<int>((total + 255) / 256);
  if (fp64)
    k_sep_sample<double><<<blocks, 256, 0, st>>>(n, lam, D, static_cast<const double*>(Z), ldz,
                                                 static_cast<double*>(Y), ldy);
  else
    k_sep_sample<float><<<blocks, 256, 0, st>>>(n, lam, D, static_cast<const float*>(Z), ldz, static_cast<float*>(Y),
                                                ldy);
  return hipGetLastError();
}

hipError_t launch_sep_cov(hipStream_t st, bool fp64, int n, int mu, const void* Y, int ldy, const int32_t* order,
                          const double* w, const double* pc, double c1, double cmu, double* C, int ldc,
                          const DevScalars* sc) {
  if (fp64)
    k_sep_cov<double><<<ceil_div(n, 256), 256, 0, st>>>(n, mu, static_cast<const double*>(Y), ldy, order, w, pc, c1,
                                                        cmu, C, ldc, sc);
  else
    k_sep_cov<float><<<ceil_div(n, 256), 256, 0, st>>>(n, mu, static_cast<const float*>(Y), ldy, order, w, pc, c1,
                                                       cmu, C, ldc, sc);
  return hipGetLastError();
}

hipError_t launch_sep_eigen(hipStream_t st, bool fp64, int n, const double* C, int ldc, double* D, void* BD, int ldbd,
                            DevScalars* sc) {
  if (fp64)
    k_sep_eigen<double><<<1, 256, 0, st>>>(n, C, ldc, D, static_cast<double*>(BD), ldbd, sc);
  else
    k_sep_eigen<float><<<1, 256, 0, st>>>(n, C, ldc, D, static_cast<float*>(BD), ldbd, sc);
  return hipGetLastError();
}

hipError_t launch_polar_step(hipStream_t st, int n, double* B, int ldb, const double* T, int ldt) {
  const int64_t total = static_cast<int64_t>(n) * n;
  k_polar_step<<<static_cast<int>((total + 255) / 256), 256, 0, st>>>(n, B, ldb, T, ldt);
  return hipGetLastError();
}

hipError_t launch_set_identity(hipStream_t st, double* A, int n, int ld) {
  const int64_t total = static_cast<int64_t>(n) * ld;
  k_set_identity<<<static_cast<int>((total + 255) / 256), 256, 0, st>>>(A, n, ld);
  return hipGetLastError();
}

hipError_t launch_to_precision(hipStream_t st, bool fp64, const double* src, int ld_src, void* dst, int ld_dst,
                               int rows, int cols) {
  const int64_t total = static_cast<int64_t>(rows) * cols;
  const int blocks = static_cast<int>((total + 255) / 256);
  if (blocks == 0) return hipSuccess;
  if (fp64)
    k_convert<double><<<blocks, 256, 0, st>>>(src, ld_src, static_cast<double*>(dst), ld_dst, rows, cols);
  else
    k_convert<float><<<blocks, 256, 0, st>>>(src, ld_src, static_cast<float*>(dst), ld_dst, rows, cols);
  return hipGetLastError();
}

}  // namespace cmx
