// Float64 eigendecomposition C = B D^2 B^T (Sec. 2.1; the O(n^3) step that
// the paper hands to LAPACK dsyev in Sec. 3.1), as a warm-started parallel
// two-sided block Jacobi method.
//
//  1. Warm start: A = B_old^T C B_old with the previous eigenvectors, which is
//     nearly diagonal because C moves little per generation.  (B_old = I on
//     the first call of a descent.)
//  2. A (padded to N = 32 k with zero rows / columns, which no rotation ever
//     touches) is cut into p = N/16 blocks of 16 indices.  A sweep runs p-1
//     rounds of a round-robin tournament over the blocks; in each round the
//     p/2 disjoint block pairs (I, J) are handled at once:
//       R1: one cyclic Jacobi sweep (Golub & Van Loan, sym.schur2 rotations)
//           over the 32 x 32 matrix S = A[{I,J},{I,J}] in LDS gives an
//           orthogonal Q_IJ;
//       R2: every 32 x 32 tile of A is replaced by Q_P1^T A_tile Q_P2 (lower
//           tiles computed, upper mirrored) and V[:, {I,J}] <- V[:, {I,J}] Q_IJ.
//     Sweeps stop when the off-diagonal Frobenius norm of A falls below
//     1e-13 of its total norm.
//  3. B = B_old V, D = sqrt(diag A), then the pairs are canonicalised like the
//     oracle: ascending eigenvalues, each column's largest-magnitude entry
//     positive.  B D is also written in the sampling precision.
#include <vector>

#include "internal.h"

namespace cmx {

namespace {

constexpr int kNB = 16;          // indices per block
constexpr int kS = 2 * kNB;      // pair problem size
constexpr int kLD = kS + 1;      // LDS row stride (bank-conflict padding)
constexpr double kOffTol = 1e-13;

typedef double doublex4 __attribute__((ext_vector_type(4)));

// 1/x and 1/sqrt(x) from the hardware approximations (about 1e-7 relative)
// refined by two Newton steps to full double precision.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

// Jacobi rotation J = [[c, s], [-s, c]] on (a, b) with (J^T S J)_ab = 0
// (Golub & Van Loan, sym.schur2): t = sign(delta) 2 d / (|delta| + sqrt(delta^2 + 4 d^2))
// with delta = S_bb - S_aa, d = S_ab; c = 1/sqrt(1 + t^2), s = t c.
__device__ __forceinline__ void jacobi_rotation(double saa, double sbb, double d, double thr, double& c,
                                                double& s) {
  c = 1.0;
  s = 0.0;
  if (!(fabs(d) > thr)) return;
  const double delta = sbb - saa;
  const double h2 = fma(delta, delta, 4.0 * d * d);
  const double h = h2 * rsq_nr(h2);
  const double t = (delta >= 0.0 ? 2.0 : -2.0) * d * rcp_nr(fabs(delta) + h);
  c = rsq_nr(fma(t, t, 1.0));
  s = t * c;
}

// round-robin (circle method) pairing of `p` players, round r, pair k
__device__ __forceinline__ void rr_pair(int p, int r, int k, int& a, int& b) {
  if (k == 0) {
    a = p - 1;
    b = r;
  } else {
    a = (r + k) % (p - 1);
    b = (r - k + (p - 1)) % (p - 1);
  }
}

// global index of local index l (0..31) of the pair made of blocks (I, J)
__device__ __forceinline__ int gidx(int I, int J, int l) { return l < kNB ? I * kNB + l : J * kNB + (l - kNB); }

__device__ __forceinline__ void block_pair(int p, int round, int P, int& I, int& J) {
  int a, b;
  rr_pair(p, round, P, a, b);
  I = min(a, b);
  J = max(a, b);
}

// R1: one cyclic Jacobi sweep over S = A[{I,J},{I,J}] for each pair of this
// round, accumulating Q.  Each thread owns one 2x2 block (pair x, pair y) of
// the 16 disjoint rotations of an inner round and recomputes the two
// rotations it needs (sym.schur2) instead of waiting for them, so an inner
// round costs one read phase and one write phase.
__global__ void __launch_bounds__(256) k_jac_pair(const double* __restrict__ A, int N, int p, int round,
                                                  const double* __restrict__ scale, double* __restrict__ Qg,
                                                  int inner_sweeps) {
  __shared__ double S[kS * kLD];
  __shared__ double Q[kS * kLD];
  const int P = blockIdx.x;
  int I, J;
  block_pair(p, round, P, I, J);
  const int t = threadIdx.x;
  for (int idx = t; idx < kS * kS; idx += 256) {
    const int r = idx % kS, c = idx / kS;
    S[r * kLD + c] = A[static_cast<int64_t>(gidx(I, J, c)) * N + gidx(I, J, r)];
    Q[r * kLD + c] = (r == c) ? 1.0 : 0.0;
  }
  const double thr = 2.2e-16 * (*scale);
  const int x = t % (kS / 2), y = t / (kS / 2);
  __syncthreads();
  for (int sweep = 0; sweep < inner_sweeps; ++sweep) {
    for (int rr = 0; rr < kS - 1; ++rr) {
      int ax, bx, ay, by;
      rr_pair(kS, rr, x, ax, bx);
      rr_pair(kS, rr, y, ay, by);
      const double xaa = S[ax * kLD + ax], xbb = S[bx * kLD + bx], xab = S[ax * kLD + bx];
      const double yaa = S[ay * kLD + ay], ybb = S[by * kLD + by], yab = S[ay * kLD + by];
      const double m00 = S[ax * kLD + ay], m01 = S[ax * kLD + by];
      const double m10 = S[bx * kLD + ay], m11 = S[bx * kLD + by];
      const int r0 = 2 * y, r1 = 2 * y + 1;  // the two rows of Q this thread rotates (pair x)
      const double q0a = Q[r0 * kLD + ax], q0b = Q[r0 * kLD + bx];
      const double q1a = Q[r1 * kLD + ax], q1b = Q[r1 * kLD + bx];
      __syncthreads();
      double cx, sx, cy, sy;
      jacobi_rotation(xaa, xbb, xab, thr, cx, sx);
      jacobi_rotation(yaa, ybb, yab, thr, cy, sy);
      // S_xy <- J_x^T S_xy J_y,  J = [[c, s], [-s, c]] on (a, b)
      const double r00 = m00 * cy - m01 * sy, r01 = m00 * sy + m01 * cy;
      const double r10 = m10 * cy - m11 * sy, r11 = m10 * sy + m11 * cy;
      double n00 = cx * r00 - sx * r10, n01 = cx * r01 - sx * r11;
      double n10 = sx * r00 + cx * r10, n11 = sx * r01 + cx * r11;
      if (x == y) {  // the annihilated entry is exactly zero
        n01 = 0.0;
        n10 = 0.0;
      }
      S[ax * kLD + ay] = n00;
      S[ax * kLD + by] = n01;
      S[bx * kLD + ay] = n10;
      S[bx * kLD + by] = n11;
      // Q <- Q J_x on rows r0, r1
      Q[r0 * kLD + ax] = cx * q0a - sx * q0b;
      Q[r0 * kLD + bx] = sx * q0a + cx * q0b;
      Q[r1 * kLD + ax] = cx * q1a - sx * q1b;
      Q[r1 * kLD + bx] = sx * q1a + cx * q1b;
      __syncthreads();
    }
  }
  double* q = Qg + static_cast<int64_t>(P) * kS * kS;
  for (int idx = t; idx < kS * kS; idx += 256) q[idx] = Q[(idx % kS) * kLD + idx / kS];  // column-major
}

// 32x32x32 product on the float64 matrix cores: wave w (of 4) computes the
// 16x16 block (w & 1, w >> 1) of  OUT = op(L) * R,  op(L) = L or L^T, all
// operands in LDS with row stride kLD.
template <bool LT>
__device__ __forceinline__ void mm32(const double* Lm, const double* Rm, double* Out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int bi = w & 1, bj = w >> 1;
  const int li = lane & 15, lk = lane >> 4;
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < kS; k0 += 4) {
    const int k = k0 + lk;
    const double a = LT ? Lm[k * kLD + bi * 16 + li] : Lm[(bi * 16 + li) * kLD + k];
    const double b = Rm[k * kLD + bj * 16 + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Out[(bi * 16 + lk + 4 * r) * kLD + bj * 16 + li] = acc[r];
}

// R2: A tiles (P1 >= P2) <- Q_P1^T A Q_P2 (mirrored), V chunks <- V Q_P.
__global__ void __launch_bounds__(256) k_jac_apply(double* __restrict__ A, double* __restrict__ V, int N, int p,
                                                   int round, const double* __restrict__ Qg) {
  __shared__ double X[kS * kLD];
  __shared__ double W[kS * kLD];
  __shared__ double Q1[kS * kLD];
  __shared__ double Q2[kS * kLD];
  const int q = p / 2;
  const int ntiles = q * (q + 1) / 2;
  const int t = threadIdx.x;
  int b = blockIdx.x;
  if (b < ntiles) {
    int P1 = static_cast<int>((sqrtf(8.0f * b + 1.0f) - 1.0f) * 0.5f);
    while ((P1 + 1) * (P1 + 2) / 2 <= b) ++P1;
    while (P1 * (P1 + 1) / 2 > b) --P1;
    const int P2 = b - P1 * (P1 + 1) / 2;
    int I1, J1, I2, J2;
    block_pair(p, round, P1, I1, J1);
    block_pair(p, round, P2, I2, J2);
    const double* q1 = Qg + static_cast<int64_t>(P1) * kS * kS;
    const double* q2 = Qg + static_cast<int64_t>(P2) * kS * kS;
    for (int idx = t; idx < kS * kS; idx += 256) {
      const int r = idx % kS, c = idx / kS;
      X[r * kLD + c] = A[static_cast<int64_t>(gidx(I2, J2, c)) * N + gidx(I1, J1, r)];
      Q1[r * kLD + c] = q1[idx];
      Q2[r * kLD + c] = q2[idx];
    }
    __syncthreads();
    mm32<false>(X, Q2, W);  // W = X Q2
    __syncthreads();
    mm32<true>(Q1, W, X);   // X = Q1^T W
    __syncthreads();
    for (int idx = t; idx < kS * kS; idx += 256) {
      const int r = idx % kS, c = idx / kS;
      A[static_cast<int64_t>(gidx(I2, J2, c)) * N + gidx(I1, J1, r)] = X[r * kLD + c];
    }
    if (P1 != P2) {
      for (int idx = t; idx < kS * kS; idx += 256) {
        const int c = idx % kS, r = idx / kS;  // consecutive threads -> consecutive rows of the mirror
        A[static_cast<int64_t>(gidx(I1, J1, r)) * N + gidx(I2, J2, c)] = X[r * kLD + c];
      }
    }
    return;
  }
  b -= ntiles;
  const int P = b % q, rc = b / q;  // pair, 32-row chunk of V
  int I, J;
  block_pair(p, round, P, I, J);
  const double* qp = Qg + static_cast<int64_t>(P) * kS * kS;
  for (int idx = t; idx < kS * kS; idx += 256) {
    const int r = idx % kS, c = idx / kS;
    X[r * kLD + c] = V[static_cast<int64_t>(gidx(I, J, c)) * N + rc * kS + r];
    Q1[r * kLD + c] = qp[idx];
  }
  __syncthreads();
  mm32<false>(X, Q1, W);
  __syncthreads();
  for (int idx = t; idx < kS * kS; idx += 256) {
    const int r = idx % kS, c = idx / kS;
    V[static_cast<int64_t>(gidx(I, J, c)) * N + rc * kS + r] = W[r * kLD + c];
  }
}

// Per-column partial sums of the off-diagonal and total squared norm, and
// the column's diagonal magnitude.
__global__ void __launch_bounds__(256) k_offnorm_cols(const double* __restrict__ A, int N, int n,
                                                      double* __restrict__ part) {
  __shared__ double r1[256], r2[256];
  const int c = blockIdx.x;
  double off = 0.0, tot = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const double v = A[static_cast<int64_t>(c) * N + r];
    tot += v * v;
    if (r != c) off += v * v;
  }
  r1[threadIdx.x] = off;
  r2[threadIdx.x] = tot;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * c + 0] = r1[0];
    part[3 * c + 1] = r2[0];
    part[3 * c + 2] = fabs(A[static_cast<int64_t>(c) * N + c]);
  }
}

// flags[0] = 1 if more sweeps are needed; scale[0] = max |a_ii|
__global__ void __launch_bounds__(256) k_offnorm_final(const double* __restrict__ part, int n, int* flags,
                                                       double* scale) {
  __shared__ double r1[256], r2[256], r3[256];
  double off = 0.0, tot = 0.0, dmax = 0.0;
  for (int c = threadIdx.x; c < n; c += 256) {
    off += part[3 * c];
    tot += part[3 * c + 1];
    dmax = fmax(dmax, part[3 * c + 2]);
  }
  r1[threadIdx.x] = off;
  r2[threadIdx.x] = tot;
  r3[threadIdx.x] = dmax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
      r3[threadIdx.x] = fmax(r3[threadIdx.x], r3[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const bool finite = isfinite(r2[0]);
    flags[0] = (finite && r1[0] > kOffTol * kOffTol * r2[0]) ? 1 : 0;
    flags[1] = finite ? 0 : 1;
    scale[0] = r3[0];
  }
}

__global__ void k_fill(double* __restrict__ A, int64_t count, double v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) A[i] = v;
}

__global__ void k_identity(double* __restrict__ V, int N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < static_cast<int64_t>(N) * N) V[i] = (i / N == i % N) ? 1.0 : 0.0;
}

// eigenvalue ranks (ascending, ties by index) and positive-definiteness flag;
// the diagonal is staged through LDS in chunks
__global__ void __launch_bounds__(256) k_eig_rank(const double* __restrict__ A, int N, int n,
                                                  int32_t* __restrict__ perm, double* __restrict__ ev,
                                                  DevScalars* __restrict__ sc) {
  __shared__ double dg[1024];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double vi = i < n ? A[static_cast<int64_t>(i) * N + i] : 0.0;
  int cnt = 0;
  for (int base = 0; base < n; base += 1024) {
    const int lim = min(1024, n - base);
    for (int j = threadIdx.x; j < lim; j += 256) dg[j] = A[static_cast<int64_t>(base + j) * N + base + j];
    __syncthreads();
    for (int j = 0; j < lim; ++j) {
      const double vj = dg[j];
      cnt += (vj < vi) || (vj == vi && base + j < i);
    }
    __syncthreads();
  }
  if (i >= n) return;
  perm[cnt] = i;
  ev[i] = vi;
  if (cnt == 0) sc->eig_ok = (vi > 0.0) ? 1 : 0;
}

// sign of each column: the entry of largest magnitude (first on ties) made positive
__global__ void __launch_bounds__(256) k_colsign(const double* __restrict__ Bn, int ld, int n,
                                                 double* __restrict__ sign) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int c = blockIdx.x;
  double best = -1.0;
  int arg = 0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const double v = fabs(Bn[static_cast<int64_t>(c) * ld + r]);
    if (v > best) {
      best = v;
      arg = r;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = arg;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const int oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sign[c] = Bn[static_cast<int64_t>(c) * ld + bi[0]] < 0.0 ? -1.0 : 1.0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_permute(const double* __restrict__ Bn, int ldt, int n,
                                                 const int32_t* __restrict__ perm, const double* __restrict__ ev,
                                                 const double* __restrict__ sign, double* __restrict__ B, int ldb,
                                                 double* __restrict__ D, T* __restrict__ BD, int ldbd) {
  const int r = blockIdx.y;  // output column
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = perm[r];
  const double d = sqrt(fmax(ev[c], 0.0));
  if (row == 0) D[r] = d;
  if (row >= n) return;
  const double v = sign[c] * Bn[static_cast<int64_t>(c) * ldt + row];
  B[static_cast<int64_t>(r) * ldb + row] = v;
  BD[static_cast<int64_t>(r) * ldbd + row] = static_cast<T>(v * d);
}

}  // namespace

int eigen_solve(hipStream_t st, int n, const double* C, int ldc, double* B, int ldb, double* D, void* BD,
                bool fp64_bd, int ldbd, EigWork& w, DevScalars* sc, int max_sweeps, int* sweeps_out,
                KTimer* kt) {
  const int N = w.N;
  const int p = N / kNB;
  const int64_t NN = static_cast<int64_t>(N) * N;
  k_fill<<<static_cast<int>((NN + 255) / 256), 256, 0, st>>>(w.A, NN, 0.0);
  k_identity<<<static_cast<int>((NN + 255) / 256), 256, 0, st>>>(w.V, N);
  CMX_HIP(hipGetLastError());
  kt_begin(kt, KID_EIG_GEMM);
  CMX_HIP(launch_dgemm(st, false, false, n, n, n, C, ldc, B, ldb, w.T, ldb));   // T = C B
  kt_end(kt);
  kt_begin(kt, KID_EIG_GEMM);
  CMX_HIP(launch_dgemm(st, true, false, n, n, n, B, ldb, w.T, ldb, w.A, N));    // A = B^T T
  kt_end(kt);
  double* part = w.evals;  // 3 n doubles of scratch during the sweeps (evals has 3N)
  int host_flags[2] = {1, 0};
  int sweeps = 0;
  const int q = p / 2;
  const int apply_blocks = q * (q + 1) / 2 + (N / kS) * q;
  for (;;) {
    k_offnorm_cols<<<n, 256, 0, st>>>(w.A, N, n, part);
    k_offnorm_final<<<1, 256, 0, st>>>(part, n, w.flags, w.sign);
    CMX_HIP(hipGetLastError());
    CMX_HIP(hipMemcpyAsync(host_flags, w.flags, sizeof(host_flags), hipMemcpyDeviceToHost, st));
    CMX_HIP(hipStreamSynchronize(st));
    if (host_flags[1]) return fail(-6, "eigensolver: non-finite covariance matrix");
    if (!host_flags[0] || sweeps >= max_sweeps) break;
    for (int r = 0; r < p - 1; ++r) {
      kt_begin(kt, KID_JAC_PAIR);
      k_jac_pair<<<q, 256, 0, st>>>(w.A, N, p, r, w.sign, w.Q, 1);
      kt_end(kt);
      kt_begin(kt, KID_JAC_APPLY);
      k_jac_apply<<<apply_blocks, 256, 0, st>>>(w.A, w.V, N, p, r, w.Q);
      kt_end(kt);
    }
    CMX_HIP(hipGetLastError());
    ++sweeps;
  }
  if (sweeps_out) *sweeps_out = sweeps;
  // B_new = B V (into T), then canonical order / signs into B, D, BD
  kt_begin(kt, KID_EIG_GEMM);
  CMX_HIP(launch_dgemm(st, false, false, n, n, n, B, ldb, w.V, N, w.T, ldb));
  kt_end(kt);
  k_eig_rank<<<ceil_div(n, 256), 256, 0, st>>>(w.A, N, n, w.perm, w.evals, sc);
  k_colsign<<<n, 256, 0, st>>>(w.T, ldb, n, w.sign);
  dim3 grid(ceil_div(n, 256), n);
  if (fp64_bd)
    k_permute<double><<<grid, 256, 0, st>>>(w.T, ldb, n, w.perm, w.evals, w.sign, B, ldb, D,
                                            static_cast<double*>(BD), ldbd);
  else
    k_permute<float><<<grid, 256, 0, st>>>(w.T, ldb, n, w.perm, w.evals, w.sign, B, ldb, D,
                                           static_cast<float*>(BD), ldbd);
  CMX_HIP(hipGetLastError());
  if (host_flags[0]) return fail(-6, "eigensolver: no convergence within the sweep limit");
  return 0;
}

}  // namespace cmx
