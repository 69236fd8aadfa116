// MFMA tile GEMMs of the generation (gfx950 matrix cores).
//
//  * Sampling, Sec. 3.1 / eq. (1): Y = (B D) [z_1 .. z_lambda].  The paper's
//    m-matrix is never formed: kernels that need x use m + sigma y.
//  * Fitness: the objective terms of u = R (x - x*) = d + sigma (R y), with
//    d = R (m - x*) in float64, are reduced inside the epilogue of R * Y, so
//    the n x lambda matrix R Y never reaches HBM.  Unrotated objectives reduce
//    the terms of d + sigma y straight from Y.
//  * Covariance, eq. (3): C <- a C + c1 pc pc^T + cmu * Yhat Yhat^T with
//    Yhat = [sqrt(w_i) y_{i:lambda}] (n x mu); only lower tiles are computed
//    and the epilogue mirrors them (SYRK).
//  * FP64 products of the eigensolver (B^T C B, B V).
//
// float: v_mfma_f32_32x32x2_f32, 128x128 block tile, 4 waves of 64x64.
// double: v_mfma_f64_16x16x4_f64, 64x64 block tile, 4 waves of 32x32.
// Operands are staged through LDS in k-major layout (m / n contiguous) so
// every MFMA operand read is a conflict-free row of 32 (16) consecutive
// elements; global loads are 16-byte vectors along the contiguous dimension.
// Reductions inside epilogues run in a fixed order (no atomics), so results
// are bitwise reproducible.
#include <algorithm>

#include "internal.h"

namespace cmx {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Cfg;
// float: only the direct (unrotated) fitness reduction of the mixed paths uses
// this tile shape; their GEMMs live in the tunable float32 kernels.
template <>
struct Cfg<float> {
  static constexpr int BM = 128, BN = 128;
  using acc_t = floatx16;
};
template <>
struct Cfg<double> {
  static constexpr int BM = 64, BN = 64, BK = 16;
  static constexpr int MB = 16;
  static constexpr int KS = 4;
  static constexpr int WM = 32, WN = 32;
  static constexpr int VEC = 2;
  static constexpr int NACC = 4;
  static constexpr int PAD = 2;
  using acc_t = doublex4;
  using vec_t = double2;
  __device__ static acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // v_mfma_f64_16x16x4_f64 keeps rows lane/16, lane/16 + 4, + 8, + 12 in a lane
  __device__ static int acc_row(int r, int l) { return (l >> 4) + 4 * r; }
};

template <typename T>
__device__ __forceinline__ void vload(const T* p, T (&v)[Cfg<T>::VEC]) {
  typename Cfg<T>::vec_t x = *reinterpret_cast<const typename Cfg<T>::vec_t*>(p);
  if constexpr (Cfg<T>::VEC == 4) {
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  } else {
    v[0] = x.x; v[1] = x.y;
  }
}

// Load the (rows x BK) slab of an operand whose element (r, k) is at
//   P[r + k*ld]   (KCONTIG = false: r contiguous)   or
//   P[k + r*ld]   (KCONTIG = true:  k contiguous),
// rows r0.., k0.., into registers (2 vectors per thread), zero outside
// [0, R) x [0, K).
template <typename T, int ROWS, bool KCONTIG, int NT = 256>
struct SlabLoader {
  static constexpr int VEC = Cfg<T>::VEC, BK = Cfg<T>::BK;
  static constexpr int PASSES = ROWS * BK / VEC / NT;
  static_assert(PASSES >= 1, "slab too small for the thread count");
  T v[PASSES][VEC];

  __device__ void load(const T* __restrict__ P, int ld, int R, int K, int r0, int k0) {
    const int t = threadIdx.x;
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      int r, k;
      if constexpr (!KCONTIG) {
        constexpr int PER_COL = ROWS / VEC;
        const int q = p * NT + t;
        r = r0 + (q % PER_COL) * VEC;
        k = k0 + q / PER_COL;
        if (k < K && r + VEC <= R) {
          vload<T>(P + static_cast<int64_t>(k) * ld + r, v[p]);
        } else {
#pragma unroll
          for (int c = 0; c < VEC; ++c)
            v[p][c] = (k < K && r + c < R) ? P[static_cast<int64_t>(k) * ld + r + c] : T(0);
        }
      } else {
        constexpr int PER_ROW = BK / VEC;
        const int q = p * NT + t;
        k = k0 + (q % PER_ROW) * VEC;
        r = r0 + q / PER_ROW;
        if (r < R && k + VEC <= K) {
          vload<T>(P + static_cast<int64_t>(r) * ld + k, v[p]);
        } else {
#pragma unroll
          for (int c = 0; c < VEC; ++c)
            v[p][c] = (r < R && k + c < K) ? P[static_cast<int64_t>(r) * ld + k + c] : T(0);
        }
      }
    }
  }

  // store into LDS laid out as S[k][ROWS + PAD]
  __device__ void store(T* S) const {
    constexpr int LD = ROWS + Cfg<T>::PAD;
    const int t = threadIdx.x;
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      if constexpr (!KCONTIG) {
        constexpr int PER_COL = ROWS / VEC;
        const int q = p * NT + t;
        const int r = (q % PER_COL) * VEC, k = q / PER_COL;
#pragma unroll
        for (int c = 0; c < VEC; ++c) S[k * LD + r + c] = v[p][c];
      } else {
        constexpr int PER_ROW = BK / VEC;
        const int q = p * NT + t;
        const int k = (q % PER_ROW) * VEC, r = q / PER_ROW;
#pragma unroll
        for (int c = 0; c < VEC; ++c) S[(k + c) * LD + r] = v[p][c];
      }
    }
  }
};

// Main loop: acc[i][j] += opA(tile) * opB(tile) for one block tile (m0, n0).
// TA: A is stored K x M (element (m,k) at A[k + m*lda]); otherwise M x K.
// TB: B is stored N x K (element (k,n) at B[n + k*ldb]); otherwise K x N.
// NT = 512: two k-groups of 4 waves, waves 4-7 taking the second half of
// every k-tile into accumulators of their own (the caller folds them).
template <typename T, bool TA, bool TB, int NT = 256>
__device__ __forceinline__ void gemm_mainloop(int M, int N, int K, const T* __restrict__ A, int lda,
                                              const T* __restrict__ B, int ldb, int m0, int n0,
                                              T* As, T* Bs, typename Cfg<T>::acc_t (&acc)[2][2]) {
  using C = Cfg<T>;
  constexpr int LDA = C::BM + C::PAD, LDB = C::BN + C::PAD;
  constexpr int KG = NT / 256;
  static_assert(C::BK % (KG * C::KS) == 0, "k-tile must split evenly over the k-groups");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = (wave >> 1) & 1, kg = wave >> 2;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < C::NACC; ++r) acc[i][j][r] = T(0);

  SlabLoader<T, C::BM, TA, NT> la;   // TA -> k contiguous in memory
  SlabLoader<T, C::BN, !TB, NT> lb;  // !TB -> k contiguous in memory
  const int nk = (K + C::BK - 1) / C::BK;
  if (nk == 0) return;
  la.load(A, lda, M, K, m0, 0);
  lb.load(B, ldb, N, K, n0, 0);
  la.store(As);
  lb.store(Bs);
  __syncthreads();
  const int kidx = lane / C::MB, midx = lane % C::MB;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) {
      la.load(A, lda, M, K, m0, (kt + 1) * C::BK);
      lb.load(B, ldb, N, K, n0, (kt + 1) * C::BK);
    }
#pragma unroll
    for (int k2 = 0; k2 < C::BK / KG; k2 += C::KS) {
      const int kk = kg * (C::BK / KG) + k2;
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[(kk + kidx) * LDA + wm * C::WM + i * C::MB + midx];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[(kk + kidx) * LDB + wn * C::WN + j * C::MB + midx];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = C::mfma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
    if (kt + 1 < nk) {
      la.store(As);
      lb.store(Bs);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- epilogues

template <typename T>
struct EpiStore {
  T* C;
  int ldc;
  __device__ void operator()(const typename Cfg<T>::acc_t (&acc)[2][2], int M, int N, int m0, int n0,
                             T*) const {
    using Cf = Cfg<T>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = n0 + wn * Cf::WN + j * Cf::MB + lane % Cf::MB;
        if (col >= N) continue;
#pragma unroll
        for (int r = 0; r < Cf::NACC; ++r) {
          const int row = m0 + wm * Cf::WM + i * Cf::MB + Cf::acc_row(r, lane);
          if (row < M) C[static_cast<int64_t>(col) * ldc + row] = acc[i][j][r];
        }
      }
  }
};

// objective term of one coordinate; Rastrigin uses the identity
// 10 - 10 cos(2 pi u) = 20 sin^2(pi u), which keeps full relative accuracy
// near the optimum where the cosine form cancels.
template <typename T>
__device__ __forceinline__ T objective_term(int kind, T u, T coef) {
  if (kind == 3) {
    T s;
    if constexpr (sizeof(T) == 4) s = sinpif(u); else s = sinpi(u);
    return u * u + T(20) * s * s;
  }
  if (kind == 2) return coef * u * u;
  return u * u;
}

template <typename T>
struct EpiFitness {
  int kind;
  const double* d;
  const T* coef;
  const DevScalars* sc;
  T* partial;
  int ldp;
  __device__ void operator()(const typename Cfg<T>::acc_t (&acc)[2][2], int M, int N, int m0, int n0,
                             T* smem) const {
    using Cf = Cfg<T>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const T sigma = static_cast<T>(sc->sigma);
    T s[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      T sum = T(0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < Cf::NACC; ++r) {
          const int row = m0 + wm * Cf::WM + i * Cf::MB + Cf::acc_row(r, lane);
          if (row < M) {
            const T u = static_cast<T>(d[row]) + sigma * acc[i][j][r];
            sum += objective_term<T>(kind, u, kind == 2 ? coef[row] : T(1));
          }
        }
      // lanes sharing a column hold different row groups: fold them in a fixed order
      if constexpr (Cf::MB == 32) {
        sum += __shfl_xor(sum, 32);
      } else {
        sum += __shfl_xor(sum, 16);
        sum += __shfl_xor(sum, 32);
      }
      s[j] = sum;
    }
    // combine the two waves stacked along m (wm = 0, 1) through LDS
    __syncthreads();
    if (lane < Cf::MB) {
#pragma unroll
      for (int j = 0; j < 2; ++j) smem[wm * Cf::BN + wn * Cf::WN + j * Cf::MB + lane] = s[j];
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < Cf::BN) {
      const int col = n0 + t;
      if (col < N) partial[static_cast<int64_t>(m0 / Cf::BM) * ldp + col] = smem[t] + smem[Cf::BN + t];
    }
  }
};

// ------------------------------------------------------------------ kernels

template <typename T, bool TA, bool TB, class Epi>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const T* __restrict__ A, int lda,
                                              const T* __restrict__ B, int ldb, Epi epi) {
  using C = Cfg<T>;
  __shared__ T As[C::BK * (C::BM + C::PAD)];
  __shared__ T Bs[C::BK * (C::BN + C::PAD)];
  const int tiles_m = (M + C::BM - 1) / C::BM;
  const int m0 = (blockIdx.x % tiles_m) * C::BM;
  const int n0 = (blockIdx.x / tiles_m) * C::BN;
  typename C::acc_t acc[2][2];
  gemm_mainloop<T, TA, TB>(M, N, K, A, lda, B, ldb, m0, n0, As, Bs, acc);
  epi(acc, M, N, m0, n0, As);
}

// float64 C = op(A) op(B) for the eigensolver's n x n products: 64 x 64 tiles
// as two k-groups of 4 waves, so that two waves share each SIMD even when
// there is one tile per CU; k-group 1's sums are folded into waves 0-3
// through LDS (fixed order), which then store the tile.
template <bool TA, bool TB>
__global__ void __launch_bounds__(512) k_dgemm_kg(int M, int N, int K, const double* __restrict__ A, int lda,
                                                  const double* __restrict__ B, int ldb, EpiStore<double> epi) {
  using C = Cfg<double>;
  __shared__ double As[C::BK * (C::BM + C::PAD)];
  __shared__ double Bs[C::BK * (C::BN + C::PAD)];
  __shared__ double fold[4 * 4 * C::NACC * 64];
  const int tiles_m = (M + C::BM - 1) / C::BM;
  const int m0 = (blockIdx.x % tiles_m) * C::BM;
  const int n0 = (blockIdx.x / tiles_m) * C::BN;
  typename C::acc_t acc[2][2];
  gemm_mainloop<double, TA, TB, 512>(M, N, K, A, lda, B, ldb, m0, n0, As, Bs, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wq = wave & 3;
  if (wave >= 4) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < C::NACC; ++r) fold[(((r * 4 + wq) * 2 + i) * 2 + j) * 64 + lane] = acc[i][j][r];
  }
  __syncthreads();
  if (wave >= 4) return;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < C::NACC; ++r) acc[i][j][r] += fold[(((r * 4 + wq) * 2 + i) * 2 + j) * 64 + lane];
  epi(acc, M, N, m0, n0, As);
}

// two independent products of one shape in one launch (two tiles per CU at
// n ~ 1000 instead of one, so twice the waves hide the MFMA and LDS latency);
// each tile is computed exactly as by k_dgemm_kg
struct DProb {
  const double* A;
  int lda;
  const double* B;
  int ldb;
  double* C;
  int ldc;
  int K;
};
template <bool TA, bool TB>
__global__ void __launch_bounds__(512) k_dgemm_kg2(int M, int N, DProb p0, DProb p1) {
  using C = Cfg<double>;
  __shared__ double As[C::BK * (C::BM + C::PAD)];
  __shared__ double Bs[C::BK * (C::BN + C::PAD)];
  __shared__ double fold[4 * 4 * C::NACC * 64];
  const int tiles_m = (M + C::BM - 1) / C::BM, tiles = tiles_m * ((N + C::BN - 1) / C::BN);
  const int t = blockIdx.x % tiles;
  const DProb pr = blockIdx.x < tiles ? p0 : p1;
  const int m0 = (t % tiles_m) * C::BM;
  const int n0 = (t / tiles_m) * C::BN;
  typename C::acc_t acc[2][2];
  gemm_mainloop<double, TA, TB, 512>(M, N, pr.K, pr.A, pr.lda, pr.B, pr.ldb, m0, n0, As, Bs, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wq = wave & 3;
  if (wave >= 4) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < C::NACC; ++r) fold[(((r * 4 + wq) * 2 + i) * 2 + j) * 64 + lane] = acc[i][j][r];
  }
  __syncthreads();
  if (wave >= 4) return;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < C::NACC; ++r) acc[i][j][r] += fold[(((r * 4 + wq) * 2 + i) * 2 + j) * 64 + lane];
  EpiStore<double>{pr.C, pr.ldc}(acc, M, N, m0, n0, As);
}

// C[:M, :N] += W[:M, :N]
__global__ void k_add_block(double* __restrict__ Cm, int ldc, const double* __restrict__ W, int ldw, int M) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r < M) Cm[static_cast<int64_t>(c) * ldc + r] += W[static_cast<int64_t>(c) * ldw + r];
}

// the n x n product of every due descent of a group, tile for tile as
// launch_dgemm_ksplit computes it: with split, workgroups [0, tiles) the
// first K0 of k into C, [tiles, 2 tiles) the rest into W (k_dgemm_kg2);
// without, k_dgemm_kg over all of k
template <bool TA>
__global__ void __launch_bounds__(512) kg_dgemm(const GDgemm* __restrict__ g, const int* __restrict__ off, int count,
                                                GroupDueMask mask) {
  using C = Cfg<double>;
  __shared__ double As[C::BK * (C::BM + C::PAD)];
  __shared__ double Bs[C::BK * (C::BN + C::PAD)];
  __shared__ double fold[4 * 4 * C::NACC * 64];
  const int i = group_find(off, count, blockIdx.x);
  if (!due_mask_bit(mask, i)) return;
  const GDgemm& e = g[i];
  const int n = e.n, tiles_m = (n + C::BM - 1) / C::BM, tiles = tiles_m * tiles_m;
  const int w = blockIdx.x - off[i];
  const int t = w % tiles;
  const bool second = e.split && w >= tiles;
  const double* A = e.A;
  const double* B = e.B;
  int K = n;
  double* out = e.C;
  int ldo = e.ldc;
  if (e.split) {
    if (second) {
      A = TA ? e.A + e.K0 : e.A + static_cast<int64_t>(e.K0) * e.lda;
      B = e.B + e.K0;
      K = n - e.K0;
      out = e.W;
      ldo = e.ldw;
    } else {
      K = e.K0;
    }
  }
  const int m0 = (t % tiles_m) * C::BM, n0 = (t / tiles_m) * C::BN;
  typename C::acc_t acc[2][2];
  gemm_mainloop<double, TA, false, 512>(n, n, K, A, e.lda, B, e.ldb, m0, n0, As, Bs, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wq = wave & 3;
  if (wave >= 4) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < C::NACC; ++r) fold[(((r * 4 + wq) * 2 + a) * 2 + b) * 64 + lane] = acc[a][b][r];
  }
  __syncthreads();
  if (wave >= 4) return;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < C::NACC; ++r) acc[a][b][r] += fold[(((r * 4 + wq) * 2 + a) * 2 + b) * 64 + lane];
  EpiStore<double>{out, ldo}(acc, n, n, m0, n0, As);
}

// C += W for the split products of a group (ceil(n / 256) x n workgroups each)
__global__ void __launch_bounds__(256) kg_add(const GDgemm* __restrict__ g, const int* __restrict__ off, int count,
                                              GroupDueMask mask) {
  const int i = group_find(off, count, blockIdx.x);
  if (!due_mask_bit(mask, i)) return;
  const GDgemm& e = g[i];
  const int nb = (e.n + 255) / 256, w = blockIdx.x - off[i];
  const int r = (w % nb) * 256 + threadIdx.x, c = w / nb;
  if (r < e.n) e.C[static_cast<int64_t>(c) * e.ldc + r] += e.W[static_cast<int64_t>(c) * e.ldw + r];
}

__device__ __forceinline__ void lower_tile(int t, int& tm, int& tn) {
  tm = static_cast<int>((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
  while (tm * (tm + 1) / 2 > t) --tm;
  tn = t - tm * (tm + 1) / 2;
}

// Rank-mu SYRK, split over k (the mu selected points) so that the few lower
// tiles of an n x n result still fill the GPU: block (t, s) writes the partial
// product of lower tile t over k-range s into its own slot of `work`.
template <typename T>
__global__ void __launch_bounds__(256) k_syrk_part(int n, int K, int kspan, const T* __restrict__ Y,
                                                   const T* __restrict__ Y2, int ldy, T* __restrict__ work, int ntl) {
  using C = Cfg<T>;
  __shared__ T As[C::BK * (C::BM + C::PAD)];
  __shared__ T Bs[C::BK * (C::BN + C::PAD)];
  const int t = blockIdx.x % ntl, s = blockIdx.x / ntl;
  int tm, tn;
  lower_tile(t, tm, tn);
  const int k0 = s * kspan, k1 = min(K, k0 + kspan);
  typename C::acc_t acc[2][2];
  const T* Yk = Y + static_cast<int64_t>(k0) * ldy;
  const T* Yk2 = Y2 + static_cast<int64_t>(k0) * ldy;
  // A = Yhat (n x K, rows contiguous), B = Yhat2^T stored N x K -> TB (Yhat2
  // = Yhat, or its columns signed by the weights' signs)
  gemm_mainloop<T, false, true>(n, n, max(0, k1 - k0), Yk, ldy, Yk2, ldy, tm * C::BM, tn * C::BN, As, Bs, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  T* out = work + (static_cast<int64_t>(s) * ntl + t) * (C::BM * C::BN);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * C::WN + j * C::MB + lane % C::MB;
#pragma unroll
      for (int r = 0; r < C::NACC; ++r) {
        const int row = wm * C::WM + i * C::MB + C::acc_row(r, lane);
        out[col * C::BM + row] = acc[i][j][r];
      }
    }
}

// C <- a C + c1 pc pc^T + cmu * sum_s partial_s  (lower triangle, mirrored);
// the split partials are summed in ascending order.
template <typename T>
__global__ void __launch_bounds__(256) k_syrk_epi(int n, int ntl, int splits, const T* __restrict__ work,
                                                  double* __restrict__ C, int ldc, const double* __restrict__ pc,
                                                  double c1, double cmu, const DevScalars* __restrict__ sc) {
  using Cf = Cfg<T>;
  constexpr int TILE = Cf::BM * Cf::BN;
  constexpr int PER = TILE / (16 * 256);
  const int t = blockIdx.x / 16, part = blockIdx.x % 16;
  int tm, tn;
  lower_tile(t, tm, tn);
  const double a = sc->c_coef;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = (part * PER + q) * 256 + threadIdx.x;
    const int row = tm * Cf::BM + e % Cf::BM, col = tn * Cf::BN + e / Cf::BM;
    if (row >= n || col >= n || row < col) continue;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += static_cast<double>(work[(static_cast<int64_t>(s) * ntl + t) * TILE + e]);
    const int64_t at = static_cast<int64_t>(col) * ldc + row;
    const double v = a * C[at] + c1 * pc[row] * pc[col] + cmu * acc;
    C[at] = v;
    if (row != col) C[static_cast<int64_t>(row) * ldc + col] = v;
  }
}

template <typename T, bool TA, bool TB, class Epi>
hipError_t run_gemm(hipStream_t st, int M, int N, int K, const T* A, int lda, const T* B, int ldb,
                    const Epi& epi) {
  using C = Cfg<T>;
  const int tiles = ceil_div(M, C::BM) * ceil_div(N, C::BN);
  if (tiles == 0) return hipSuccess;
  k_gemm<T, TA, TB, Epi><<<tiles, 256, 0, st>>>(M, N, K, A, lda, B, ldb, epi);
  return hipGetLastError();
}

// Direct (unrotated) fitness: u = d + sigma * y read from Y, one block per
// (row tile, column tile) with the same partial layout as the GEMM epilogue.
template <typename T>
__global__ void __launch_bounds__(256) k_fitness_direct(int n, int lam, const T* __restrict__ Y, int ldy,
                                                        EpiFitness<T> epi) {
  using C = Cfg<T>;
  const int tiles_m = (n + C::BM - 1) / C::BM;
  const int m0 = (blockIdx.x % tiles_m) * C::BM;
  const int n0 = (blockIdx.x / tiles_m) * C::BN;
  // one thread per column of the tile, rows summed in ascending order
  const int t = threadIdx.x;
  if (t >= C::BN) return;
  const int col = n0 + t;
  if (col >= lam) return;
  const T sigma = static_cast<T>(epi.sc->sigma);
  const T* y = Y + static_cast<int64_t>(col) * ldy;
  T sum = T(0);
  const int mend = min(m0 + C::BM, n);
  for (int row = m0; row < mend; ++row) {
    const T u = static_cast<T>(epi.d[row]) + sigma * y[row];
    sum += objective_term<T>(epi.kind, u, epi.kind == 2 ? epi.coef[row] : T(1));
  }
  epi.partial[static_cast<int64_t>(m0 / C::BM) * epi.ldp + col] = sum;
}

template <typename T>
__device__ __forceinline__ void fitness_reduce_body(int bx, int lam, const T* __restrict__ partial, int ldp,
                                                    int tiles, double add, double* __restrict__ f) {
  const int k = bx * blockDim.x + threadIdx.x;
  if (k >= lam) return;
  double s = 0.0;
#pragma unroll 16
  for (int t = 0; t < tiles; ++t) s += static_cast<double>(partial[static_cast<int64_t>(t) * ldp + k]);
  f[k] = s + add;
}

template <typename T>
__global__ void __launch_bounds__(256) k_fitness_reduce(int lam, const T* __restrict__ partial, int ldp,
                                                        int tiles, double add, double* __restrict__ f) {
  fitness_reduce_body<T>(blockIdx.x, lam, partial, ldp, tiles, add, f);
}

__global__ void __launch_bounds__(256) kg_fitness_reduce(const GFront* __restrict__ g, const int* __restrict__ off,
                                                         int count) {
  const int i = group_find(off, count, blockIdx.x);
  const GFront& e = g[i];
  fitness_reduce_body<float>(blockIdx.x - off[i], e.lam, e.partial, e.lam, e.fit_tiles, 0.0, e.f);
}

}  // namespace

hipError_t launch_sample_gemm_f64(hipStream_t st, int n, int lam, const double* BD, int ldbd, const double* Z,
                                  int ldz, double* Y, int ldy) {
  return run_gemm<double, false, false>(st, n, lam, n, BD, ldbd, Z, ldz, EpiStore<double>{Y, ldy});
}

hipError_t launch_fitness_gemm_f64(hipStream_t st, int n, int lam, const double* R, int ldr, const double* Y, int ldy,
                                   const FitnessArgs& fa, int* row_tiles) {
  *row_tiles = ceil_div(n, Cfg<double>::BM);
  EpiFitness<double> e{fa.kind, fa.d, static_cast<const double*>(fa.coef), fa.sc,
                       static_cast<double*>(fa.partial), fa.ld_partial};
  return run_gemm<double, false, false>(st, n, lam, n, R, ldr, Y, ldy, e);
}

hipError_t launch_fitness_direct(hipStream_t st, bool fp64, int n, int lam, const void* Y, int ldy,
                                 const FitnessArgs& fa, int* row_tiles) {
  if (fp64) {
    using C = Cfg<double>;
    *row_tiles = ceil_div(n, C::BM);
    EpiFitness<double> e{fa.kind, fa.d, static_cast<const double*>(fa.coef), fa.sc,
                         static_cast<double*>(fa.partial), fa.ld_partial};
    const int tiles = *row_tiles * ceil_div(lam, C::BN);
    k_fitness_direct<double><<<tiles, 256, 0, st>>>(n, lam, static_cast<const double*>(Y), ldy, e);
  } else {
    using C = Cfg<float>;
    *row_tiles = ceil_div(n, C::BM);
    EpiFitness<float> e{fa.kind, fa.d, static_cast<const float*>(fa.coef), fa.sc,
                        static_cast<float*>(fa.partial), fa.ld_partial};
    const int tiles = *row_tiles * ceil_div(lam, C::BN);
    k_fitness_direct<float><<<tiles, 256, 0, st>>>(n, lam, static_cast<const float*>(Y), ldy, e);
  }
  return hipGetLastError();
}

hipError_t launch_fitness_reduce(hipStream_t st, bool fp64, int kind, int n, int lam,
                                 const void* partial, int ld_partial, int row_tiles, double* f) {
  (void)kind;
  (void)n;
  const int blocks = ceil_div(lam, 256);
  if (fp64)
    k_fitness_reduce<double><<<blocks, 256, 0, st>>>(lam, static_cast<const double*>(partial),
                                                     ld_partial, row_tiles, 0.0, f);
  else
    k_fitness_reduce<float><<<blocks, 256, 0, st>>>(lam, static_cast<const float*>(partial), ld_partial,
                                                    row_tiles, 0.0, f);
  return hipGetLastError();
}

void syrk_plan_f64(int n, int K, int* ntl, int* splits, int* kspan, size_t* work_elems) {
  const int bm = Cfg<double>::BM;
  const int bk = Cfg<double>::BK;
  const int tm = ceil_div(n, bm);
  *ntl = tm * (tm + 1) / 2;
  int s = ceil_div(512, *ntl);
  s = std::max(1, std::min(s, ceil_div(K, 64)));
  *kspan = round_up(ceil_div(std::max(K, 1), s), bk);
  *splits = ceil_div(std::max(K, 1), *kspan);
  *work_elems = static_cast<size_t>(*splits) * (*ntl) * bm * bm;
}

hipError_t launch_syrk_update_f64(hipStream_t st, int n, int mu, const double* Ysel, const double* Ysel2, int ldsel,
                                  double* C, int ldc, const double* pc, double c1, double cmu, const DevScalars* sc,
                                  double* work) {
  int ntl, splits, kspan;
  size_t we;
  syrk_plan_f64(n, mu, &ntl, &splits, &kspan, &we);
  k_syrk_part<double><<<ntl * splits, 256, 0, st>>>(n, mu, kspan, Ysel, Ysel2 ? Ysel2 : Ysel, ldsel, work, ntl);
  k_syrk_epi<double><<<ntl * 16, 256, 0, st>>>(n, ntl, splits, work, C, ldc, pc, c1, cmu, sc);
  return hipGetLastError();
}

hipError_t launch_dgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, const double* A, int lda,
                        const double* B, int ldb, double* C, int ldc) {
  using Cf = Cfg<double>;
  const int tiles = ceil_div(M, Cf::BM) * ceil_div(N, Cf::BN);
  if (tiles == 0) return hipSuccess;
  EpiStore<double> e{C, ldc};
  if (!ta && !tb) k_dgemm_kg<false, false><<<tiles, 512, 0, st>>>(M, N, K, A, lda, B, ldb, e);
  else if (ta && !tb) k_dgemm_kg<true, false><<<tiles, 512, 0, st>>>(M, N, K, A, lda, B, ldb, e);
  else if (!ta && tb) k_dgemm_kg<false, true><<<tiles, 512, 0, st>>>(M, N, K, A, lda, B, ldb, e);
  else k_dgemm_kg<true, true><<<tiles, 512, 0, st>>>(M, N, K, A, lda, B, ldb, e);
  return hipGetLastError();
}

hipError_t launch_group_fitness_reduce(hipStream_t st, const GFront* g, const int* off, int count, int wgs) {
  if (wgs > 0) kg_fitness_reduce<<<wgs, 256, 0, st>>>(g, off, count);
  return hipGetLastError();
}

hipError_t launch_group_dgemm(hipStream_t st, bool ta, const GDgemm* gd, const int* off_mm, int wgs_mm,
                              const int* off_add, int wgs_add, int count, const GroupDueMask& mask) {
  if (wgs_mm > 0) {
    if (ta)
      kg_dgemm<true><<<wgs_mm, 512, 0, st>>>(gd, off_mm, count, mask);
    else
      kg_dgemm<false><<<wgs_mm, 512, 0, st>>>(gd, off_mm, count, mask);
  }
  if (wgs_add > 0) kg_add<<<wgs_add, 256, 0, st>>>(gd, off_add, count, mask);
  return hipGetLastError();
}

hipError_t launch_dgemm2(hipStream_t st, int M, int N, int K, const double* A0, int lda0, const double* A1,
                         int lda1, const double* B, int ldb, double* C0, int ldc0, double* C1, int ldc1) {
  using Cf = Cfg<double>;
  const int tiles = ceil_div(M, Cf::BM) * ceil_div(N, Cf::BN);
  if (tiles == 0) return hipSuccess;
  k_dgemm_kg2<false, false><<<2 * tiles, 512, 0, st>>>(M, N, DProb{A0, lda0, B, ldb, C0, ldc0, K},
                                                      DProb{A1, lda1, B, ldb, C1, ldc1, K});
  return hipGetLastError();
}

hipError_t launch_dgemm_ksplit(hipStream_t st, bool ta, bool tb, int M, int N, int K, const double* A, int lda,
                               const double* B, int ldb, double* Cm, int ldc, double* W, int ldw) {
  using Cf = Cfg<double>;
  const int tiles = ceil_div(M, Cf::BM) * ceil_div(N, Cf::BN);
  if (tiles == 0) return hipSuccess;
  // split only while the whole product has at most one tile per CU (256 on
  // gfx950): with more tiles the CUs are already shared and the add's extra
  // pass over C costs more than the split gains
  constexpr int kCUs = 256;
  const int K0 = round_up(ceil_div(K, 2), Cf::BK);
  if (K0 >= K || tiles > kCUs) return launch_dgemm(st, ta, tb, M, N, K, A, lda, B, ldb, Cm, ldc);
  // op(A)[:, K0:] and op(B)[K0:, :]: A stored M x K (K x M if ta), B K x N (N x K if tb)
  const double* A1 = ta ? A + K0 : A + static_cast<int64_t>(K0) * lda;
  const double* B1 = tb ? B + static_cast<int64_t>(K0) * ldb : B + K0;
  const DProb p0{A, lda, B, ldb, Cm, ldc, K0}, p1{A1, lda, B1, ldb, W, ldw, K - K0};
  if (!ta && !tb) k_dgemm_kg2<false, false><<<2 * tiles, 512, 0, st>>>(M, N, p0, p1);
  else if (ta && !tb) k_dgemm_kg2<true, false><<<2 * tiles, 512, 0, st>>>(M, N, p0, p1);
  else if (!ta && tb) k_dgemm_kg2<false, true><<<2 * tiles, 512, 0, st>>>(M, N, p0, p1);
  else k_dgemm_kg2<true, true><<<2 * tiles, 512, 0, st>>>(M, N, p0, p1);
  k_add_block<<<dim3(ceil_div(M, 256), N), 256, 0, st>>>(Cm, ldc, W, ldw, M);
  return hipGetLastError();
}

}  // namespace cmx
