// Tunable float32 MFMA GEMMs of the mixed-precision generation: the sampling
// product Y = (B D) Z (eq. (1), Sec. 3.1 rewrite), the fitness product R Y with
// the objective reduced in the epilogue, and the split-k rank-mu SYRK partials
// (eq. (3)).  One kernel template, several block tiles; the tile is chosen
// per call site by the autotuner (api.hip) from kG32Configs.
//
//  * v_mfma_f32_32x32x2_f32; 4 waves in a 2 x 2 grid, each owning a
//    (BM/2) x (BN/2) sub-tile of 32 x 32 MFMA blocks;
//  * operands staged k-major in LDS (m / n contiguous, conflict-free MFMA
//    reads), double buffered, one barrier per k-tile; the next k-tile's global
//    loads (unconditional float4 reads from clamped addresses, the k-tail
//    zeroed only when staged) are in flight while the current one is
//    multiplied;
//  * XCD-aware tile order: consecutive workgroups are dispatched round-robin
//    over the 8 XCDs, so workgroup w is given tile (w mod 8) * T/8 + w / 8 and
//    each XCD walks a contiguous run of tiles that share their B columns in
//    its own L2.

#include <algorithm>

#include "internal.h"

namespace cmx {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// bijection [0, T) -> [0, T): workgroup w on XCD (w mod 8) gets the j-th tile
// of that XCD's contiguous range
__device__ __forceinline__ int xcd_swizzle(int w, int T) {
  const int x = w & 7, j = w >> 3;
  const int q = T >> 3, r = T & 7;
  return x * q + min(x, r) + j;
}

// NT threads: 4 waves per k-group, KG = NT / 256 k-groups.  With KG = 2 the
// waves 4-7 multiply the second half of every k-tile into accumulators of
// their own (the caller folds the two groups).
template <int BM, int BN, int BK, bool TB, int NT = 256>
struct G32 {
  // B staged k-major from k-contiguous columns (!TB) is written one float per
  // k: a row stride of BN + 2 words puts the 4 k-rows a half-wave writes on
  // disjoint banks (BN + 4 would fold rows 0 and 2 together); float4 staging
  // (TB, and A) needs a stride that keeps 16-byte alignment
  static constexpr int LDA = BM + 4, LDB = TB ? BN + 4 : BN + 2;
  static constexpr int TMB = BM / 64, TNB = BN / 64;  // 32x32 blocks per wave
  static constexpr int KG = NT / 256;
  static constexpr int A_V4 = BM * BK / 4 / NT;       // float4 loads per thread
  static constexpr int B_V4 = BN * BK / 4 / NT;
  static_assert(A_V4 >= 1 && B_V4 >= 1, "tile too small for the thread count");
  static_assert(BK % (2 * KG) == 0, "k-tile must split evenly over the k-groups");
  float4 ra[A_V4], rb[B_V4];

  // Operand loads are branch free.  Every operand is stored with a leading
  // dimension that is a multiple of 4 and at least its row count rounded up
  // to 4, so a float4 that starts inside a column stays inside it.  Rows past
  // the tile's edge (m >= M, n >= N) are clamped into the last float4 of the
  // column: they load values that only reach output rows / columns past the
  // edge, which no epilogue stores.  Entries past the reduction length K are
  // read from a clamped address and replaced by zero when they are staged in
  // LDS, so the loads of the next k-tile stay in flight over the current
  // tile's MFMAs.
  __device__ static float4 zero_unless(float4 v, bool ok) {
    return make_float4(ok ? v.x : 0.0f, ok ? v.y : 0.0f, ok ? v.z : 0.0f, ok ? v.w : 0.0f);
  }

  // A: M x K column-major (m contiguous)
  __device__ void load_a(const float* __restrict__ A, int lda, int K, int m0, int k0) {
    constexpr int PER_COL = BM / 4;
#pragma unroll
    for (int p = 0; p < A_V4; ++p) {
      const int q = p * NT + threadIdx.x;
      const int m = min(m0 + (q % PER_COL) * 4, lda - 4), k = k0 + q / PER_COL;
      ra[p] = *reinterpret_cast<const float4*>(A + static_cast<int64_t>(min(k, K - 1)) * lda + m);
    }
  }
  __device__ void store_a(float* S, int K, int k0) const {
    constexpr int PER_COL = BM / 4;
#pragma unroll
    for (int p = 0; p < A_V4; ++p) {
      const int q = p * NT + threadIdx.x;
      *reinterpret_cast<float4*>(&S[(q / PER_COL) * LDA + (q % PER_COL) * 4]) =
          zero_unless(ra[p], k0 + q / PER_COL < K);
    }
  }
  // B: K x N column-major (k contiguous) when !TB, else element (k, n) at B[n + k ldb]
  __device__ void load_b(const float* __restrict__ B, int ldb, int N, int K, int n0, int k0) {
#pragma unroll
    for (int p = 0; p < B_V4; ++p) {
      const int q = p * NT + threadIdx.x;
      if constexpr (!TB) {
        constexpr int PER_ROW = BK / 4;
        const int k = k0 + (q % PER_ROW) * 4, n = min(n0 + q / PER_ROW, N - 1);
        rb[p] = *reinterpret_cast<const float4*>(B + static_cast<int64_t>(n) * ldb + min(k, ldb - 4));
      } else {
        constexpr int PER_COL = BN / 4;
        const int n = min(n0 + (q % PER_COL) * 4, ldb - 4), k = k0 + q / PER_COL;
        rb[p] = *reinterpret_cast<const float4*>(B + static_cast<int64_t>(min(k, K - 1)) * ldb + n);
      }
    }
  }
  __device__ void store_b(float* S, int K, int k0) const {
#pragma unroll
    for (int p = 0; p < B_V4; ++p) {
      const int q = p * NT + threadIdx.x;
      if constexpr (!TB) {
        constexpr int PER_ROW = BK / 4;
        const int k = (q % PER_ROW) * 4, n = q / PER_ROW, kk = k0 + k;
        S[(k + 0) * LDB + n] = kk < K ? rb[p].x : 0.0f;
        S[(k + 1) * LDB + n] = kk + 1 < K ? rb[p].y : 0.0f;
        S[(k + 2) * LDB + n] = kk + 2 < K ? rb[p].z : 0.0f;
        S[(k + 3) * LDB + n] = kk + 3 < K ? rb[p].w : 0.0f;
      } else {
        constexpr int PER_COL = BN / 4;
        *reinterpret_cast<float4*>(&S[(q / PER_COL) * LDB + (q % PER_COL) * 4]) =
            zero_unless(rb[p], k0 + q / PER_COL < K);
      }
    }
  }

  // 32x32 block (i, j) of this wave lies strictly above the tile's diagonal
  __device__ static bool upper_block(int wm, int wn, int i, int j) {
    return wm * (BM / 2) + i * 32 < wn * (BN / 2) + j * 32;
  }

  // acc += A[m0.., k-range] * B[k-range, n0..] for k in [0, K).  Without MMA
  // the wave only stages operands (it takes part in the loads and barriers of
  // its workgroup) and acc stays zero.
  template <bool MMA = true>
  __device__ void mainloop(int N, int K, const float* __restrict__ A, int lda, const float* __restrict__ B, int ldb,
                           int m0, int n0, float* As, float* Bs, floatx16 (&acc)[TMB][TNB]) {
    // the wave index is uniform; readfirstlane lets the compiler keep it scalar
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave & 1, wn = (wave >> 1) & 1, kg = wave >> 2;
#pragma unroll
    for (int i = 0; i < TMB; ++i)
#pragma unroll
      for (int j = 0; j < TNB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int nk = (K + BK - 1) / BK;
    if (nk == 0) return;
    load_a(A, lda, K, m0, 0);
    load_b(B, ldb, N, K, n0, 0);
    store_a(As, K, 0);
    store_b(Bs, K, 0);
    __syncthreads();
    const int kidx = lane >> 5, midx = lane & 31;
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      const float* Ac = As + cur * BK * LDA;
      const float* Bc = Bs + cur * BK * LDB;
      if (kt + 1 < nk) {
        load_a(A, lda, K, m0, (kt + 1) * BK);
        load_b(B, ldb, N, K, n0, (kt + 1) * BK);
      }
#pragma unroll
      for (int k2 = 0; k2 < BK / KG; k2 += 2) {
        const int kk = kg * (BK / KG) + k2;
        if constexpr (MMA) {
          float a[TMB], b[TNB];
#pragma unroll
          for (int i = 0; i < TMB; ++i) a[i] = Ac[(kk + kidx) * LDA + wm * (BM / 2) + i * 32 + midx];
#pragma unroll
          for (int j = 0; j < TNB; ++j) b[j] = Bc[(kk + kidx) * LDB + wn * (BN / 2) + j * 32 + midx];
#pragma unroll
          for (int i = 0; i < TMB; ++i)
#pragma unroll
            for (int j = 0; j < TNB; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
      }
      if (kt + 1 < nk) {
        store_a(As + (cur ^ 1) * BK * LDA, K, (kt + 1) * BK);
        store_b(Bs + (cur ^ 1) * BK * LDB, K, (kt + 1) * BK);
      }
      __syncthreads();
    }
  }
};

// row of accumulator element r held by lane l (column l % 32) of a 32x32 block
__device__ __forceinline__ int acc_row(int r, int l) { return (r >> 2) * 8 + (l >> 5) * 4 + (r & 3); }

template <int BM, int BN>
struct Epi32Store {
  float* Y;
  int ldy;
  __device__ void operator()(const floatx16 (&acc)[BM / 64][BN / 64], int M, int N, int m0, int n0, float*) const {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;
#pragma unroll
    for (int i = 0; i < BM / 64; ++i)
#pragma unroll
      for (int j = 0; j < BN / 64; ++j) {
        const int col = n0 + wn * (BN / 2) + j * 32 + (lane & 31);
        if (col >= N) continue;
        const int rbase = m0 + wm * (BM / 2) + i * 32 + (lane >> 5) * 4;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int row = rbase + g * 8;
          float* dst = Y + static_cast<int64_t>(col) * ldy + row;
          if (row + 4 <= M) {
            *reinterpret_cast<float4*>(dst) = make_float4(acc[i][j][4 * g], acc[i][j][4 * g + 1],
                                                          acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]);
          } else {
            for (int c = 0; c < 4 && row + c < M; ++c) dst[c] = acc[i][j][4 * g + c];
          }
        }
      }
  }
};

// objective term; Rastrigin via 10 - 10 cos(2 pi u) = 20 sin^2(pi u)
__device__ __forceinline__ float obj_term(int kind, float u, float coef) {
  if (kind == 3) {
    const float s = sinpif(u);
    return u * u + 20.0f * s * s;
  }
  if (kind == 2) return coef * u * u;
  return u * u;
}

template <int BM, int BN>
struct Epi32Fitness {
  int kind;
  const double* d;
  const float* coef;
  const DevScalars* sc;
  float* partial;
  int ldp;
  __device__ void operator()(const floatx16 (&acc)[BM / 64][BN / 64], int M, int N, int m0, int n0,
                             float* smem) const {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const float sigma = static_cast<float>(sc->sigma);
    float s[BN / 64];
#pragma unroll
    for (int j = 0; j < BN / 64; ++j) {
      float sum = 0.0f;
#pragma unroll
      for (int i = 0; i < BM / 64; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = m0 + wm * (BM / 2) + i * 32 + acc_row(r, lane);
          if (row < M) {
            const float u = static_cast<float>(d[row]) + sigma * acc[i][j][r];
            sum += obj_term(kind, u, kind == 2 ? coef[row] : 1.0f);
          }
        }
      sum += __shfl_xor(sum, 32);  // the other 4-row groups of the same column
      s[j] = sum;
    }
    __syncthreads();
    if (lane < 32) {
#pragma unroll
      for (int j = 0; j < BN / 64; ++j) smem[wm * BN + wn * (BN / 2) + j * 32 + lane] = s[j];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < BN; t += 256) {
      const int col = n0 + t;
      if (col < N) partial[static_cast<int64_t>(m0 / BM) * ldp + col] = smem[t] + smem[BN + t];
    }
  }
};

template <int BM, int BN, int BK, bool TB, class Epi>
__device__ __forceinline__ void g32_body(int bid, int M, int N, int K, const float* __restrict__ A, int lda,
                                         const float* __restrict__ B, int ldb, const Epi& epi, float* As,
                                         float* Bs) {
  using G = G32<BM, BN, BK, TB>;
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  const int tile = xcd_swizzle(bid, tiles_m * tiles_n);
  const int m0 = (tile % tiles_m) * BM, n0 = (tile / tiles_m) * BN;
  floatx16 acc[G::TMB][G::TNB];
  G g;
  g.mainloop(N, K, A, lda, B, ldb, m0, n0, As, Bs, acc);
  epi(acc, M, N, m0, n0, As);
}

template <int BM, int BN, int BK, bool TB, class Epi>
__global__ void __launch_bounds__(256) k_g32(int M, int N, int K, const float* __restrict__ A, int lda,
                                             const float* __restrict__ B, int ldb, Epi epi) {
  using G = G32<BM, BN, BK, TB>;
  __shared__ float As[2 * BK * G::LDA];
  __shared__ float Bs[2 * BK * G::LDB];
  g32_body<BM, BN, BK, TB, Epi>(blockIdx.x, M, N, K, A, lda, B, ldb, epi, As, Bs);
}

// the sampling product (SITE = G32_SAMPLE: Y = (B D) Z) or the fitness product
// with its objective epilogue (G32_FITNESS: R Y) of every descent of a group
template <int BM, int BN, int BK, int SITE>
__global__ void __launch_bounds__(256) kg_g32(const GFront* __restrict__ g, const int* __restrict__ off, int count) {
  using G = G32<BM, BN, BK, false>;
  __shared__ float As[2 * BK * G::LDA];
  __shared__ float Bs[2 * BK * G::LDB];
  const int i = group_find(off, count, blockIdx.x);
  const GFront& e = g[i];
  const int bid = blockIdx.x - off[i];
  if constexpr (SITE == G32_SAMPLE) {
    g32_body<BM, BN, BK, false>(bid, e.n, e.lam, e.n, e.BD, e.ldn, e.Z, e.ldn, Epi32Store<BM, BN>{e.Y, e.ldn}, As,
                                Bs);
  } else {
    const Epi32Fitness<BM, BN> epi{e.kind, e.d, e.coef, e.sc, e.partial, e.lam};
    g32_body<BM, BN, BK, false>(bid, e.n, e.lam, e.n, e.Rt, e.ldn, e.Y, e.ldn, epi, As, Bs);
  }
}

__device__ __forceinline__ void lower_tile(int t, int& tm, int& tn) {
  tm = static_cast<int>((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
  while (tm * (tm + 1) / 2 > t) --tm;
  tn = t - tm * (tm + 1) / 2;
}

// rank-mu SYRK partials: workgroup (tile t, split s) writes its lower tile's
// partial product over k-range s into work[(s ntl + t) BM^2 ...].  With
// NT = 512 the two k-groups of waves are folded through LDS first, so a
// workgroup covers twice the k-range per partial tile written.
template <int BM, int BK, int NT>
__device__ __forceinline__ void syrk32_body(int bid, int nwg, int n, int K, int kspan, const float* __restrict__ Y,
                                            const float* __restrict__ Y2, int ldy, float* __restrict__ work, int ntl,
                                            float* smem) {
  using G = G32<BM, BM, BK, true, NT>;
  float* As = smem;
  float* Bs = smem + 2 * BK * G::LDA;
  const int item = xcd_swizzle(bid, nwg);
  const int t = item % ntl, s = item / ntl;
  int tm, tn;
  lower_tile(t, tm, tn);
  const int k0 = s * kspan, k1 = min(K, k0 + kspan);
  floatx16 acc[G::TMB][G::TMB];
  const float* Yk = Y + static_cast<int64_t>(k0) * ldy;
  const float* Yk2 = Y2 + static_cast<int64_t>(k0) * ldy;
  G g;
  const bool diag = tm == tn;
  // on a diagonal tile the wave whose whole sub-tile lies above the diagonal
  // (rows [0, BM/2), columns [BM/2, BM)) multiplies nothing: its SIMD is free
  // for the other resident workgroups' waves
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (diag && (wv & 3) == 2)
    g.template mainloop<false>(n, max(0, k1 - k0), Yk, ldy, Yk2, ldy, tm * BM, tn * BM, As, Bs, acc);
  else
    g.template mainloop<true>(n, max(0, k1 - k0), Yk, ldy, Yk2, ldy, tm * BM, tn * BM, As, Bs, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if constexpr (G::KG == 2) {
    // k-group 1 hands its sums to k-group 0 (lane-contiguous, conflict free)
    static_assert(4 * G::TMB * G::TMB * 64 * 16 <= 2 * BK * (G::LDA + G::LDB), "fold buffer exceeds LDS");
    const int wq = wave & 3;
    if (wave >= 4) {
#pragma unroll
      for (int i = 0; i < G::TMB; ++i)
#pragma unroll
        for (int j = 0; j < G::TMB; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) smem[(((r * 4 + wq) * G::TMB + i) * G::TMB + j) * 64 + lane] = acc[i][j][r];
    }
    __syncthreads();
    if (wave >= 4) return;
#pragma unroll
    for (int i = 0; i < G::TMB; ++i)
#pragma unroll
      for (int j = 0; j < G::TMB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] += smem[(((r * 4 + wq) * G::TMB + i) * G::TMB + j) * 64 + lane];
  }
  // fragment-native layout: each lane stores its 16 accumulator values
  // contiguously, so a wave writes one contiguous 4 KiB run per 32x32 block.
  // Blocks above a diagonal tile's diagonal are never read back.
  float* out = work + (static_cast<int64_t>(s) * ntl + t) * (BM * BM);
#pragma unroll
  for (int i = 0; i < G::TMB; ++i)
#pragma unroll
    for (int j = 0; j < G::TMB; ++j) {
      if (diag && G::upper_block(wave & 1, wave >> 1, i, j)) continue;
      float4* dst = reinterpret_cast<float4*>(out + ((((wave * G::TMB + i) * G::TMB + j) * 64 + lane) << 4));
#pragma unroll
      for (int q = 0; q < 4; ++q)
        dst[q] = make_float4(acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]);
    }
}

template <int BM, int BK, int NT>
__global__ void __launch_bounds__(NT) k_syrk32(int n, int K, int kspan, const float* __restrict__ Y,
                                               const float* __restrict__ Y2, int ldy, float* __restrict__ work,
                                               int ntl) {
  using G = G32<BM, BM, BK, true, NT>;
  __shared__ float smem[2 * BK * G::LDA + 2 * BK * G::LDB];
  syrk32_body<BM, BK, NT>(blockIdx.x, static_cast<int>(gridDim.x), n, K, kspan, Y, Y2, ldy, work, ntl, smem);
}

template <int BM, int BK, int NT>
__global__ void __launch_bounds__(NT) kg_syrk32(const GFront* __restrict__ g, const int* __restrict__ off, int count) {
  using G = G32<BM, BM, BK, true, NT>;
  __shared__ float smem[2 * BK * G::LDA + 2 * BK * G::LDB];
  const int i = group_find(off, count, blockIdx.x);
  const GFront& e = g[i];
  syrk32_body<BM, BK, NT>(blockIdx.x - off[i], e.syrk_ntl * e.syrk_splits, e.n, e.mu, e.syrk_kspan, e.Ysel, e.Ysel,
                          e.ldn, e.syrk_work, e.syrk_ntl, smem);
}

// C <- a C + c1 pc pc^T + cmu * sum_s partial_s, one workgroup per 32 x 32
// block (R, Q) of the lower block triangle (R >= Q, in units of 32 rows).  The
// block is one contiguous 4 KiB run of every split's partial tile (fragment-
// native layout above); wavefront g of the workgroup takes the 16-byte group g
// of each lane's 16 values, so one 16-byte load per split and lane, and up to
// eight splits are in flight at once.  Each value is summed in float64 in
// ascending split order.  The sums pass through LDS so that both the block and
// its mirror are written as whole columns of C.
template <int BM>
__device__ __forceinline__ void syrk32_epi_body(int bid, int n, int ntl, int splits, const float* __restrict__ work,
                                                double* __restrict__ C, int ldc, const double* __restrict__ pc,
                                                double c1, double cmu, const DevScalars* __restrict__ sc, double* T) {
  constexpr int H = BM / 2, TB = BM / 64, PB = BM / 32;
  constexpr int U = 8;  // splits per batch of loads
  int R, Q;
  lower_tile(bid, R, Q);
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int tm = R / PB, tn = Q / PB;
  const int t = tm * (tm + 1) / 2 + tn;
  const int rl = (R % PB) * 32, cl = (Q % PB) * 32;  // block origin inside its tile
  const int wave = rl / H + 2 * (cl / H);
  const int i = (rl % H) >> 5, j = (cl % H) >> 5;
  const float4* src = reinterpret_cast<const float4*>(
      work + static_cast<int64_t>(t) * (BM * BM) + ((((wave * TB + i) * TB + j) * 64 + lane) << 4)) + g;
  const int64_t sstride = static_cast<int64_t>(ntl) * (BM * BM / 4);  // in float4
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int s = 0;
  for (; s + U <= splits; s += U) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[(s + u) * sstride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[0] += static_cast<double>(v[u].x);
      acc[1] += static_cast<double>(v[u].y);
      acc[2] += static_cast<double>(v[u].z);
      acc[3] += static_cast<double>(v[u].w);
    }
  }
  for (; s < splits; ++s) {
    const float4 v = src[s * sstride];
    acc[0] += static_cast<double>(v.x);
    acc[1] += static_cast<double>(v.y);
    acc[2] += static_cast<double>(v.z);
    acc[3] += static_cast<double>(v.w);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) T[(lane & 31) * 33 + acc_row(4 * g + r, lane)] = acc[r];
  __syncthreads();
  const double a = sc->c_coef;
  const int r0 = R * 32, q0 = Q * 32;
  const int row = threadIdx.x & 31, sub = threadIdx.x >> 5;  // 8 columns per pass
  // the block, column by column
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    const int col = 8 * cc + sub;
    const int gr = r0 + row, gc = q0 + col;
    if (gr < n && gc < n && (R != Q || row >= col)) {
      const int64_t at = static_cast<int64_t>(gc) * ldc + gr;
      const double v = a * C[at] + c1 * pc[gr] * pc[gc] + cmu * T[col * 33 + row];
      C[at] = v;
      T[col * 33 + row] = v;
    }
  }
  __syncthreads();
  // the mirror: element (row, col) of the block goes to C(q0 + col, r0 + row)
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int brow = 8 * rr + sub, bcol = threadIdx.x & 31;
    const int gr = r0 + brow, gc = q0 + bcol;
    if (gr < n && gc < n && (R != Q || brow > bcol))
      C[static_cast<int64_t>(gr) * ldc + gc] = T[bcol * 33 + brow];
  }
}

template <int BM>
__global__ void __launch_bounds__(256) k_syrk32_epi(int n, int ntl, int splits, const float* __restrict__ work,
                                                    double* __restrict__ C, int ldc, const double* __restrict__ pc,
                                                    double c1, double cmu, const DevScalars* __restrict__ sc) {
  __shared__ double T[32 * 33];
  syrk32_epi_body<BM>(blockIdx.x, n, ntl, splits, work, C, ldc, pc, c1, cmu, sc, T);
}

template <int BM>
__global__ void __launch_bounds__(256) kg_syrk32_epi(const GFront* __restrict__ g, const int* __restrict__ off,
                                                     int count) {
  __shared__ double T[32 * 33];
  const int i = group_find(off, count, blockIdx.x);
  const GFront& e = g[i];
  syrk32_epi_body<BM>(blockIdx.x - off[i], e.n, e.syrk_ntl, e.syrk_splits, e.syrk_work, e.C, e.ldn, e.pc, e.kp.c1,
                      e.kp.cmu, e.sc, T);
}

template <int BM, int BN, int BK>
hipError_t launch_group_cfg(hipStream_t st, int site, const GFront* g, const int* off, int count, int wgs) {
  if (wgs == 0) return hipSuccess;
  if (site == G32_SAMPLE)
    kg_g32<BM, BN, BK, G32_SAMPLE><<<wgs, 256, 0, st>>>(g, off, count);
  else
    kg_g32<BM, BN, BK, G32_FITNESS><<<wgs, 256, 0, st>>>(g, off, count);
  return hipGetLastError();
}

template <int BM, int BK, int NT>
hipError_t launch_group_syrk_cfg(hipStream_t st, const GFront* g, const int* off_syrk, int wgs_syrk,
                                 const int* off_epi, int wgs_epi, int count) {
  if (wgs_syrk > 0) kg_syrk32<BM, BK, NT><<<wgs_syrk, NT, 0, st>>>(g, off_syrk, count);
  if (wgs_epi > 0) kg_syrk32_epi<BM><<<wgs_epi, 256, 0, st>>>(g, off_epi, count);
  return hipGetLastError();
}

template <int BM, int BN, int BK>
hipError_t launch_cfg(hipStream_t st, int site, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                      void* out, int ldo, const G32FitArgs* fa, KTimer* kt, int kid) {
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles == 0) return hipSuccess;
  if (site == G32_SAMPLE) {
    timed_launch(kt, kid, k_g32<BM, BN, BK, false, Epi32Store<BM, BN>>, tiles, 256, st, M, N, K, A, lda, B, ldb,
                 Epi32Store<BM, BN>{static_cast<float*>(out), ldo});
  } else {
    Epi32Fitness<BM, BN> e{fa->kind, fa->d, fa->coef, fa->sc, static_cast<float*>(out), ldo};
    timed_launch(kt, kid, k_g32<BM, BN, BK, false, Epi32Fitness<BM, BN>>, tiles, 256, st, M, N, K, A, lda, B, ldb,
                 e);
  }
  return hipGetLastError();
}

template <int BM, int BK, int NT>
hipError_t launch_syrk_cfg(hipStream_t st, int cfg, int n, int K, const float* Y, const float* Y2, int ldy,
                           float* work, double* C, int ldc, const double* pc, double c1, double cmu,
                           const DevScalars* sc, bool partial_only, KTimer* kt) {
  int ntl, splits, kspan;
  size_t we;
  syrk32_plan(cfg, n, K, &ntl, &splits, &kspan, &we);
  timed_launch(kt, KID_SYRK, k_syrk32<BM, BK, NT>, ntl * splits, NT, st, n, K, kspan, Y, Y2 ? Y2 : Y, ldy, work,
               ntl);
  if (!partial_only) {
    const int nb = (n + 31) / 32;
    timed_launch(kt, KID_SYRK_EPI, k_syrk32_epi<BM>, nb * (nb + 1) / 2, 256, st, n, ntl, splits, work, C, ldc, pc,
                 c1, cmu, sc);
  }
  return hipGetLastError();
}

}  // namespace

// block tiles (BM x BN x BK) the tuner chooses from; SYRK uses the square ones
const G32Config kG32Configs[kG32NumConfigs] = {
    {128, 128, 16}, {128, 64, 16}, {64, 128, 16}, {256, 128, 16}, {128, 128, 32}, {64, 64, 32}, {64, 64, 16},
};

// threads per workgroup of the SYRK products of square configuration cfg:
// 128 x 128 x 32 runs as two k-groups of 4 waves
int syrk32_threads(int cfg) { return cfg == 4 ? 512 : 256; }

// split-k plan: at most as many workgroups as are resident at once on 256 CUs
// (two 4-wave 128-tile workgroups, one 8-wave one, or four 64-tile ones per
// CU), k-ranges a multiple of 32
void syrk32_plan(int cfg, int n, int K, int* ntl, int* splits, int* kspan, size_t* work_elems) {
  const int bm = kG32Configs[cfg].bm;
  const int tm = ceil_div(n, bm);
  *ntl = tm * (tm + 1) / 2;
  const int target = syrk32_threads(cfg) == 512 ? 256 : (bm == 64 ? 1024 : 512);
  int s = target / *ntl;
  s = std::max(1, std::min(s, ceil_div(K, 64)));
  *kspan = round_up(ceil_div(std::max(K, 1), s), 32);
  *splits = ceil_div(std::max(K, 1), *kspan);
  *work_elems = static_cast<size_t>(*splits) * (*ntl) * bm * bm;
}

size_t syrk32_max_work(int n, int K) {
  size_t best = 0;
  for (int c = 0; c < kG32NumConfigs; ++c) {
    if (!g32_config_valid(c, G32_SYRK)) continue;
    int ntl, splits, kspan;
    size_t we;
    syrk32_plan(c, n, K, &ntl, &splits, &kspan, &we);
    best = std::max(best, we);
  }
  return best;
}

bool g32_config_valid(int cfg, int site) {
  if (cfg < 0 || cfg >= kG32NumConfigs) return false;
  if (site == G32_SYRK) return kG32Configs[cfg].bm == kG32Configs[cfg].bn;
  return true;
}

int g32_row_tiles(int cfg, int M) { return ceil_div(M, kG32Configs[cfg].bm); }

hipError_t g32_gemm(hipStream_t st, int cfg, int site, int M, int N, int K, const float* A, int lda, const float* B,
                    int ldb, void* out, int ldo, const G32FitArgs* fa, KTimer* kt, int kid) {
  switch (cfg) {
    case 0: return launch_cfg<128, 128, 16>(st, site, M, N, K, A, lda, B, ldb, out, ldo, fa, kt, kid);
    case 1: return launch_cfg<128, 64, 16>(st, site, M, N, K, A, lda, B, ldb, out, ldo, fa, kt, kid);
    case 2: return launch_cfg<64, 128, 16>(st, site, M, N, K, A, lda, B, ldb, out, ldo, fa, kt, kid);
    case 3: return launch_cfg<256, 128, 16>(st, site, M, N, K, A, lda, B, ldb, out, ldo, fa, kt, kid);
    case 4: return launch_cfg<128, 128, 32>(st, site, M, N, K, A, lda, B, ldb, out, ldo, fa, kt, kid);
    case 5: return launch_cfg<64, 64, 32>(st, site, M, N, K, A, lda, B, ldb, out, ldo, fa, kt, kid);
    case 6: return launch_cfg<64, 64, 16>(st, site, M, N, K, A, lda, B, ldb, out, ldo, fa, kt, kid);
    default: return hipErrorInvalidValue;
  }
}

int g32_tiles(int cfg, int M, int N) { return ceil_div(M, kG32Configs[cfg].bm) * ceil_div(N, kG32Configs[cfg].bn); }

void syrk32_group_wgs(int cfg, int n, int K, int* wgs_products, int* wgs_epi) {
  int ntl, splits, kspan;
  size_t we;
  syrk32_plan(cfg, n, K, &ntl, &splits, &kspan, &we);
  const int nb = (n + 31) / 32;
  *wgs_products = ntl * splits;
  *wgs_epi = nb * (nb + 1) / 2;
}

hipError_t launch_group_g32(hipStream_t st, int cfg, int site, const GFront* g, const int* off, int count, int wgs) {
  switch (cfg) {
    case 0: return launch_group_cfg<128, 128, 16>(st, site, g, off, count, wgs);
    case 1: return launch_group_cfg<128, 64, 16>(st, site, g, off, count, wgs);
    case 2: return launch_group_cfg<64, 128, 16>(st, site, g, off, count, wgs);
    case 3: return launch_group_cfg<256, 128, 16>(st, site, g, off, count, wgs);
    case 4: return launch_group_cfg<128, 128, 32>(st, site, g, off, count, wgs);
    case 5: return launch_group_cfg<64, 64, 32>(st, site, g, off, count, wgs);
    case 6: return launch_group_cfg<64, 64, 16>(st, site, g, off, count, wgs);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_group_syrk(hipStream_t st, int cfg, const GFront* g, const int* off_syrk, int wgs_syrk,
                             const int* off_epi, int wgs_epi, int count) {
  switch (cfg) {
    case 0: return launch_group_syrk_cfg<128, 16, 256>(st, g, off_syrk, wgs_syrk, off_epi, wgs_epi, count);
    case 4: return launch_group_syrk_cfg<128, 32, 512>(st, g, off_syrk, wgs_syrk, off_epi, wgs_epi, count);
    case 5: return launch_group_syrk_cfg<64, 32, 256>(st, g, off_syrk, wgs_syrk, off_epi, wgs_epi, count);
    case 6: return launch_group_syrk_cfg<64, 16, 256>(st, g, off_syrk, wgs_syrk, off_epi, wgs_epi, count);
    default: return hipErrorInvalidValue;
  }
}

hipError_t g32_syrk(hipStream_t st, int cfg, int n, int K, const float* Y, const float* Y2, int ldy, float* work,
                    double* C, int ldc, const double* pc, double c1, double cmu, const DevScalars* sc,
                    bool partial_only, KTimer* kt) {
  switch (cfg) {
    case 0:
      return launch_syrk_cfg<128, 16, 256>(st, 0, n, K, Y, Y2, ldy, work, C, ldc, pc, c1, cmu, sc, partial_only, kt);
    case 4:
      return launch_syrk_cfg<128, 32, 512>(st, 4, n, K, Y, Y2, ldy, work, C, ldc, pc, c1, cmu, sc, partial_only, kt);
    case 5:
      return launch_syrk_cfg<64, 32, 256>(st, 5, n, K, Y, Y2, ldy, work, C, ldc, pc, c1, cmu, sc, partial_only, kt);
    case 6:
      return launch_syrk_cfg<64, 16, 256>(st, 6, n, K, Y, Y2, ldy, work, C, ldc, pc, c1, cmu, sc, partial_only, kt);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cmx
