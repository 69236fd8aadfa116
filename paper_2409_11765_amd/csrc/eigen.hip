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
//       R1: on the 32 x 32 matrix S = A[{I,J},{I,J}] in LDS, 16 inner rounds
//           of 16 disjoint Jacobi rotations (Golub & Van Loan, sym.schur2)
//           over the cross pairs (i in I, j in J) give an orthogonal Q_IJ;
//           the first round of a sweep also rotates the pairs inside each
//           block, so every index pair is rotated once per sweep;
//       R2: every 32 x 32 tile of A is replaced by Q_P1^T A_tile Q_P2 (lower
//           tiles computed, upper mirrored) and V[:, {I,J}] <- V[:, {I,J}] Q_IJ.
//     R1 is a chain of dependent rotation rounds (latency bound) and R2 is a
//     wide, bandwidth bound update, so one launch per round does both: the
//     R2 of round r (A ping-pongs between two buffers) and, in q extra
//     workgroups, the R1 of round r+1, each of which recomputes the three
//     16 x 16 round-r blocks its next pair needs instead of waiting for them.
//     Rotation angles are formed in float32 (they only set how far an entry
//     is reduced); cosines and sines are float64 and orthogonal to rounding.
//     Sweeps stop when the off-diagonal Frobenius norm of A falls below
//     1e-13 of its total norm (summed per tile by the last round); once it
//     is below 1e-8, a closing correction (below) takes the last sweep's place.
//     V starts as B_old, so the rotations land straight in B = B_old V.
//  3. D = sqrt(diag A), then the pairs are canonicalised like the
//     oracle: ascending eigenvalues, each column's largest-magnitude entry
//     positive.  B D is also written in the sampling precision.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <vector>

#include "internal.h"

namespace cmx {

namespace {

constexpr int kNB = 16;          // indices per block
constexpr int kS = 2 * kNB;      // pair problem size
constexpr int kLD = kS + 1;      // LDS row stride (bank-conflict padding)
constexpr double kOffTol = 1e-13;
// closing correction: queued once off(A) <= kCorrOff ||A||_F, applied only if
// the angles satisfy ||Theta||_F <= EigWork::corr_max_theta (at most 2e-3)
constexpr double kCorrOff = 1e-8;
constexpr int kMaxCorrections = 4;  // per solve

typedef double doublex4 __attribute__((ext_vector_type(4)));

// Jacobi rotation J = [[c, s], [-s, c]] on (a, b) that annihilates (J^T S J)_ab
// up to the accuracy of t (Golub & Van Loan, sym.schur2): t = sign(delta) 2 d /
// (|delta| + sqrt(delta^2 + 4 d^2)) with delta = S_bb - S_aa, d = S_ab;
// c = 1/sqrt(1 + t^2), s = t c; the identity when |d| <= thr.
// t only decides how far the entry is reduced, so it is formed in float32 from
// the entries scaled by inv = 1/max|a_ii| (relative error ~1e-7: the entry
// drops to ~1e-7 of itself and later rotations remove the rest).  c is then
// refined to float64 precision from that t by two Newton steps, because
// c^2 (1 + t^2) = 1 is what keeps each rotation, and so Q, orthogonal.
// Branch free, so the callers' loads issue up front and two rotations
// interleave.
__device__ __forceinline__ void jacobi_rotation(double saa, double sbb, double d, double thr, double inv, double& c,
                                                double& s) {
  const double dd = fabs(d) > thr ? d : 0.0;
  const float df = static_cast<float>(dd * inv);
  const float delta = static_cast<float>((sbb - saa) * inv);
  const float h = __builtin_amdgcn_sqrtf(fmaf(delta, delta, 4.0f * df * df));
  // |delta| + h >= 2 |df| > 0 whenever df != 0; the floor only guards 0 / 0
  const float tf = (delta >= 0.0f ? 2.0f : -2.0f) * df * __builtin_amdgcn_rcpf(fmaxf(fabsf(delta) + h, 1e-30f));
  const double t = static_cast<double>(tf);
  const double x = fma(t, t, 1.0);
  double y = static_cast<double>(__builtin_amdgcn_rsqf(fmaf(tf, tf, 1.0f)));
  y = y * fma(-0.5 * x * y, y, 1.5);
  c = y * fma(-0.5 * x * y, y, 1.5);
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

// the pair of round r that contains block X (inverse of rr_pair)
__device__ __forceinline__ int pair_of(int p, int r, int X) {
  if (X == p - 1 || X == r) return 0;
  const int d = (X - r + (p - 1)) % (p - 1);
  return d <= p / 2 - 1 ? d : (p - 1) - d;
}

// 16x16 output block of a product with inner dimension 32 on the float64
// matrix cores (8 steps of v_mfma_f64_16x16x4f64).  Lane l supplies
// A(i = l & 15, k = 4 s + (l >> 4)) in a[s] and B(k = 4 s + (l >> 4), j = l & 15)
// in b[s]; the result holds OUT(row = (l >> 4) + 4 r, col = l & 15) in acc[r].
__device__ __forceinline__ doublex4 mfma_k32(const double (&a)[8], const double (&b)[8]) {
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 8; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
  return acc;
}

// 32x32 column-major matrix q (global) into LDS rows: Q[row * kLD + col]
__device__ __forceinline__ void load_q(const double* __restrict__ q, double* Q) {
#pragma unroll
  for (int k = 0; k < kS * kS / 256; ++k) {
    const int idx = threadIdx.x + 256 * k;
    Q[(idx % kS) * kLD + idx / kS] = q[idx];
  }
}

// Rotation x (0..15) of inner round r as branch-free index arithmetic (see
// inner_pair): INTRA = round-robin inside each 16-block, else cross pairs.
template <bool INTRA>
__device__ __forceinline__ void pair_idx(int r, int x, int& a, int& b) {
  if constexpr (INTRA) {
    const int k = x & 7, off = (x >> 3) * kNB;
    int u = r + k;
    u = u >= kNB - 1 ? u - (kNB - 1) : u;
    int v = r - k;
    v = v < 0 ? v + (kNB - 1) : v;
    a = (k == 0 ? kNB - 1 : u) + off;
    b = (k == 0 ? r : v) + off;
  } else {
    a = x;
    b = kNB + ((x + r) & (kNB - 1));
  }
}

// Value held by lane 0 of this lane's 16-lane row (DPP row broadcast, two
// 32-bit moves).
__device__ __forceinline__ double row_lane0(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), 0x150, 0xF, 0xF, false);  // row_newbcast:0
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x150, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Value held by lane (lane + 1) mod 16 of this lane's 16-lane row (DPP
// row_ror:15, two 32-bit moves).
__device__ __forceinline__ double row_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), 0x12F, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x12F, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// One cross inner round (rotation x pairs a = x with b = 16 + (x + rr) mod 16)
// with the thread's four Q entries in registers (qa0, qa1 = Q[2y, a],
// Q[2y + 1, a]; qb0, qb1 = Q[2y, b], Q[2y + 1, b]) and two of its four S
// entries: m00 = S[x, y], which no other thread reads unless x = y (then it
// is also stored, for rotation x), and m10 = S[b, y], which next round
// belongs to lane (lane + 1) mod 16 of the row.  S[x, b_y] and S[b, b_y] go
// through LDS.  Otherwise as inner_round below.
__device__ __forceinline__ void inner_round_cross(const double* S, double* Sn, double thr, double inv, int rr, int x,
                                                  int y, double& qa0, double& qa1, double& qb0, double& qb1,
                                                  double& m00, double& m10) {
  int ax, bx, ay, by;
  pair_idx<false>(rr, x, ax, bx);
  pair_idx<false>(rr, y, ay, by);
  const double xaa = S[ax * kLD + ax], xbb = S[bx * kLD + bx], xab = S[ax * kLD + bx];
  const double m01 = S[ax * kLD + by], m11 = S[bx * kLD + by];
  double cx, sx;
  jacobi_rotation(xaa, xbb, xab, thr, inv, cx, sx);
  const double cy = row_lane0(cx), sy = row_lane0(sx);
  const double p00 = m00 * cy - m01 * sy, p01 = m00 * sy + m01 * cy;
  const double p10 = m10 * cy - m11 * sy, p11 = m10 * sy + m11 * cy;
  const double n00 = cx * p00 - sx * p10, n11 = sx * p01 + cx * p11;
  const double n01 = cx * p01 - sx * p11, n10 = sx * p00 + cx * p10;
  if (x == y) Sn[ax * kLD + ay] = n00;  // the diagonal, read by rotation x's threads
  Sn[ax * kLD + by] = n01;
  Sn[bx * kLD + by] = n11;
  m00 = n00;
  m10 = n10;
  const double a0 = cx * qa0 - sx * qb0, b0 = sx * qa0 + cx * qb0;
  const double a1 = cx * qa1 - sx * qb1, b1 = sx * qa1 + cx * qb1;
  qa0 = a0;
  qb0 = b0;
  qa1 = a1;
  qb1 = b1;
}

// One inner round (INTRA: the round-robin pairs inside each 16-block, with Q
// in LDS): every thread owns one 2x2 block (rotation x, rotation y),
// computes rotation x and takes rotation y from lane 0 of its 16-lane row
// (the caller lays the threads out so that a row shares y and its lane 0
// has x = y), updates its block of S into the other buffer and rows r0, r1
// of Q for rotation x.
template <bool INTRA>
__device__ __forceinline__ void inner_round(const double* S, double* Sn, double* Q, double thr, double inv, int rr,
                                            int x, int y) {
  int ax, bx, ay, by;
  pair_idx<INTRA>(rr, x, ax, bx);
  pair_idx<INTRA>(rr, y, ay, by);
  const int r0 = 2 * y, r1 = 2 * y + 1;
  const double xaa = S[ax * kLD + ax], xbb = S[bx * kLD + bx], xab = S[ax * kLD + bx];
  const double m00 = S[ax * kLD + ay], m01 = S[ax * kLD + by];
  const double m10 = S[bx * kLD + ay], m11 = S[bx * kLD + by];
  const double q0a = Q[r0 * kLD + ax], q0b = Q[r0 * kLD + bx];
  const double q1a = Q[r1 * kLD + ax], q1b = Q[r1 * kLD + bx];
  double cx, sx;
  jacobi_rotation(xaa, xbb, xab, thr, inv, cx, sx);
  const double cy = row_lane0(cx), sy = row_lane0(sx);
  // S_xy <- J_x^T S_xy J_y,  J = [[c, s], [-s, c]] on (a, b)
  const double p00 = m00 * cy - m01 * sy, p01 = m00 * sy + m01 * cy;
  const double p10 = m10 * cy - m11 * sy, p11 = m10 * sy + m11 * cy;
  // (for x == y, n01 = n10 is what remains of the annihilated entry)
  const double n00 = cx * p00 - sx * p10, n11 = sx * p01 + cx * p11;
  const double n01 = cx * p01 - sx * p11, n10 = sx * p00 + cx * p10;
  Sn[ax * kLD + ay] = n00;
  Sn[ax * kLD + by] = n01;
  Sn[bx * kLD + ay] = n10;
  Sn[bx * kLD + by] = n11;
  // Q <- Q J_x on rows r0, r1 (only this thread touches these entries this round)
  Q[r0 * kLD + ax] = cx * q0a - sx * q0b;
  Q[r0 * kLD + bx] = sx * q0a + cx * q0b;
  Q[r1 * kLD + ax] = cx * q1a - sx * q1b;
  Q[r1 * kLD + bx] = sx * q1a + cx * q1b;
}

// R1 on S (LDS, buffer S0; S1 is its double buffer): the rotations of one
// outer round (optionally the 15 intra-block rounds, then the 16 cross
// rounds), accumulated into Q (LDS) and written column-major to qout.  One
// barrier per inner round.  A block made of padding indices only (>= n) has
// zero rows and columns in S, so every rotation that involves it is exactly
// the identity (t = 0, c = 1, s = 0): with pad_j (block J is padding) the
// cross rounds are skipped, with pad_i (both blocks) the intra rounds too.
__device__ void rotate_pair(double* S0, double* S1, double* Q, double thr, double inv, bool with_intra,
                            double* __restrict__ qout, bool pad_i = false, bool pad_j = false) {
  const int t = threadIdx.x;
  for (int idx = t; idx < kS * kS; idx += 256) Q[(idx % kS) * kLD + idx / kS] = (idx % kS == idx / kS) ? 1.0 : 0.0;
  // a row of 16 lanes shares y; x = (lane + y) mod 16, so lane 0 of the row
  // computes rotation y
  const int y = t / (kS / 2), x = ((t & 15) + y) & 15;
  double* Sa = S0;
  double* Sb = S1;
  __syncthreads();
  if (with_intra && !pad_i) {
    for (int rr = 0; rr < kNB - 1; ++rr) {
      inner_round<true>(Sa, Sb, Q, thr, inv, rr, x, y);
      double* tmp = Sa;
      Sa = Sb;
      Sb = tmp;
      __syncthreads();
    }
  }
  // cross rounds: the thread's Q entries (rows 2y, 2y + 1; columns a = x and
  // b) and S entries S[x, y], S[b, y] stay in registers; the next round's b
  // entries are the ones lane (lane + 1) mod 16 of the row holds now
  const int r0 = 2 * y, r1 = 2 * y + 1;
  double qa0 = Q[r0 * kLD + x], qa1 = Q[r1 * kLD + x];
  double qb0 = Q[r0 * kLD + kNB + x], qb1 = Q[r1 * kLD + kNB + x];
  double m00 = Sa[x * kLD + y], m10 = Sa[(kNB + x) * kLD + y];
  for (int rr = 0; rr < (pad_j ? 0 : kNB); ++rr) {
    inner_round_cross(Sa, Sb, thr, inv, rr, x, y, qa0, qa1, qb0, qb1, m00, m10);
    double* tmp = Sa;
    Sa = Sb;
    Sb = tmp;
    if (rr + 1 < kNB) {
      qb0 = row_next(qb0);
      qb1 = row_next(qb1);
      m10 = row_next(m10);
    }
    __syncthreads();
  }
  {
    const int b = pad_j ? kNB + x : kNB + ((x + kNB - 1) & (kNB - 1));
    Q[r0 * kLD + x] = qa0;
    Q[r1 * kLD + x] = qa1;
    Q[r0 * kLD + b] = qb0;
    Q[r1 * kLD + b] = qb1;
  }
  __syncthreads();
  if (qout)
    for (int idx = t; idx < kS * kS; idx += 256) qout[idx] = Q[(idx % kS) * kLD + idx / kS];
  __syncthreads();
}

// First pair solves of a descent's eigensolve: round 0 (with the intra-block
// rotations) straight from A.
__device__ __forceinline__ void jac_first_body(int P, const double* __restrict__ A, int N, int n, int p,
                                               const double* __restrict__ scale, double* __restrict__ Qg,
                                               double* lds) {
  double* S0 = lds;
  double* S1 = lds + kS * kLD;
  double* Q = lds + 2 * kS * kLD;
  int I, J;
  block_pair(p, 0, P, I, J);
  for (int idx = threadIdx.x; idx < kS * kS; idx += 256) {
    const int r = idx % kS, c = idx / kS;
    S0[r * kLD + c] = A[static_cast<int64_t>(gidx(I, J, c)) * N + gidx(I, J, r)];
  }
  __syncthreads();
  const double sc = *scale;
  rotate_pair(S0, S1, Q, 2.2e-16 * sc, sc > 0.0 ? 1.0 / sc : 0.0, true, Qg + static_cast<int64_t>(P) * kS * kS,
              I * kNB >= n, J * kNB >= n);
}

__global__ void __launch_bounds__(256) k_jac_first(const double* __restrict__ A, int N, int n, int p,
                                                   const double* __restrict__ scale, double* __restrict__ Qg) {
  __shared__ double lds[3 * kS * kLD];
  jac_first_body(blockIdx.x, A, N, n, p, scale, Qg, lds);
}

// One outer round r: workgroups [0, q) run the pair solves of the next round
// (r + 1, or round 0 of the next sweep after the last round); workgroups
// [q, q + q(q+1)/2) write the round-r lower tiles Q_P1^T A_cur Q_P2 of A into
// A_next (and their mirrors) and the tiles' off-diagonal / total squared norms
// into tilepart; the rest update 32-row pieces of V with V Q_P.  MFMA operands
// that come from A or V are loaded from global memory straight into the
// fragment registers; only the Q's and cross-wave intermediates go through LDS.
// Stores of the round's outputs (A_next, V) as relaxed device-scope atomic
// stores: they are written through the XCD's L2 (cache policy sc1), so a round
// leaves no dirty L2 lines behind and the end-of-kernel cache flush before the
// next dependent launch has almost nothing to write back.  The values and
// their order are those of plain stores; the next launch reads them after the
// kernel boundary.
__device__ __forceinline__ void store_through(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kLU = kNB + 1;                           // row stride of the 32 x 16 stage-1 products
constexpr int kRoundLds = 3 * kS * kLD + 3 * kS * kLU;  // doubles of LDS per workgroup

__device__ __forceinline__ void jac_round_body(int b, const double* __restrict__ Acur, double* __restrict__ Anext,
                                               double* __restrict__ V, const double* __restrict__ Qcur,
                                               double* __restrict__ Qnext, int N, int n, int r,
                                               const double* __restrict__ scale, double* __restrict__ tilepart,
                                               double* lds) {
  const int p = N / kNB, q = p / 2;
  const int ntiles = q * (q + 1) / 2;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (b < q) {
    // ---- pair solve of the next round.  Its 32 x 32 problem S is made of
    // three 16 x 16 blocks of the round-r output, recomputed here from A_cur
    // and the round-r Q's instead of waited for:
    //   S11 = Qa[:, ca]^T Xa Qa[:, ca],  S22 = Qb[:, cb]^T Xb Qb[:, cb],
    //   S12 = Qa[:, ca]^T Xab Qb[:, cb]
    // (Xa, Xb, Xab: round-r tiles of A_cur; ca / cb: the 16 columns of the
    // round-r pair that become the next pair's blocks).  Stage 1 forms the
    // 32 x 16 products U = X Q[:, c] (6 MFMA blocks over the 4 waves),
    // stage 2 the three 16 x 16 blocks.
    const bool wrap = (r + 1 == p - 1);
    const int rn = wrap ? 0 : r + 1;
    int In, Jn;
    block_pair(p, rn, b, In, Jn);
    const int Pa = pair_of(p, r, In), Pb = pair_of(p, r, Jn);
    int Ia, Ja, Ib, Jb;
    block_pair(p, r, Pa, Ia, Ja);
    block_pair(p, r, Pb, Ib, Jb);
    const bool same = (Pa == Pb);  // p = 2: both blocks from one round-r pair
    const int ca = (In == Ia) ? 0 : kNB;
    const int cb = same ? ((Jn == Ia) ? 0 : kNB) : ((Jn == Ib) ? 0 : kNB);
    double* Qa = lds;
    double* Qb = lds + kS * kLD;
    double* S = lds + 2 * kS * kLD;
    double* U = lds + 3 * kS * kLD;  // 3 x [32][kLU]
    // stage-1 blocks: 2u + h = rows [16h, 16h + 16) of U_u; u = 0: Xa Qa[:, ca],
    // 1: Xb Qb[:, cb], 2: Xab Qb[:, cb] (U_2 = U_1 when same)
    const int nblk = same ? 4 : 6;
    double fa[2][8];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int blk = w + 4 * v;
      if (blk < nblk) {  // uniform per wave
        const int u = blk >> 1, R = (blk & 1) * kNB;
        const int rI = u == 1 ? Ib : Ia, rJ = u == 1 ? Jb : Ja;
        const int cI = u == 0 ? Ia : Ib, cJ = u == 0 ? Ja : Jb;
        const int row = gidx(rI, rJ, R + li);
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) fa[v][s2] = Acur[static_cast<int64_t>(gidx(cI, cJ, 4 * s2 + lk)) * N + row];
      }
    }
    load_q(Qcur + static_cast<int64_t>(Pa) * kS * kS, Qa);
    load_q(Qcur + static_cast<int64_t>(Pb) * kS * kS, Qb);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int blk = w + 4 * v;
      if (blk < nblk) {
        const int u = blk >> 1, R = (blk & 1) * kNB;
        const double* Qs = u == 0 ? Qa : Qb;
        const int c = u == 0 ? ca : cb;
        double bq[8];
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) bq[s2] = Qs[(4 * s2 + lk) * kLD + c + li];
        const doublex4 acc = mfma_k32(fa[v], bq);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) U[u * kS * kLU + (R + lk + 4 * rr) * kLU + li] = acc[rr];
      }
    }
    __syncthreads();
    if (w < 3) {
      // wave 0: S11 = Qa[:, ca]^T U_0; 1: S22 = Qb[:, cb]^T U_1; 2: S12 = Qa[:, ca]^T U_2
      const double* Ql = w == 1 ? Qb : Qa;
      const int c = w == 1 ? cb : ca;
      const int u = (w == 2 && same) ? 1 : w;
      double aq[8], bu[8];
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) {
        aq[s2] = Ql[(4 * s2 + lk) * kLD + c + li];
        bu[s2] = U[u * kS * kLU + (4 * s2 + lk) * kLU + li];
      }
      const doublex4 acc = mfma_k32(aq, bu);
      const int ro = w == 1 ? kNB : 0, co = w == 0 ? 0 : kNB;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        S[(ro + lk + 4 * rr) * kLD + co + li] = acc[rr];
        if (w == 2) S[(kNB + li) * kLD + lk + 4 * rr] = acc[rr];
      }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(2);  // the pair solves are the round's critical path
    const double sc = *scale;
    rotate_pair(S, Qa, Qb, 2.2e-16 * sc, sc > 0.0 ? 1.0 / sc : 0.0, wrap,
                Qnext + static_cast<int64_t>(b) * kS * kS, In * kNB >= n, Jn * kNB >= n);
    return;
  }
  b -= q;
  if (b < ntiles) {
    // ---- round-r tile T = Q1^T X Q2 (X = A_cur[rows of pair P1, cols of pair P2])
    // of A_next.  Stage 1: W = X Q2.  Stage 2 forms both T and T^T so that the
    // tile and its mirror are each stored by 16-lane runs of consecutive rows.
    int P1 = static_cast<int>((sqrtf(8.0f * b + 1.0f) - 1.0f) * 0.5f);
    while ((P1 + 1) * (P1 + 2) / 2 <= b) ++P1;
    while (P1 * (P1 + 1) / 2 > b) --P1;
    const int P2 = b - P1 * (P1 + 1) / 2;
    int I1, J1, I2, J2;
    block_pair(p, r, P1, I1, J1);
    block_pair(p, r, P2, I2, J2);
    double* Q1 = lds;
    double* Q2 = lds + kS * kLD;
    double* W = lds + 2 * kS * kLD;
    double* red = lds + 3 * kS * kLD;
    const int bi = w & 1, bj = w >> 1;
    double fx[8];
    {
      const int row = gidx(I1, J1, bi * kNB + li);
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) fx[s2] = Acur[static_cast<int64_t>(gidx(I2, J2, 4 * s2 + lk)) * N + row];
    }
    load_q(Qcur + static_cast<int64_t>(P1) * kS * kS, Q1);
    load_q(Qcur + static_cast<int64_t>(P2) * kS * kS, Q2);
    __syncthreads();
    {
      double bq[8];
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) bq[s2] = Q2[(4 * s2 + lk) * kLD + bj * kNB + li];
      const doublex4 acc = mfma_k32(fx, bq);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) W[(bi * kNB + lk + 4 * rr) * kLD + bj * kNB + li] = acc[rr];
    }
    __syncthreads();
    // M1 = T^T = W^T Q1 (block (bi, bj)): row j, col i -> A_next(gidx1(i), gidx2(j))
    // M2 = T   = Q1^T W (block (bi, bj)): row i, col j -> A_next(gidx2(j), gidx1(i))
    double a1[8], b1[8], a2[8], b2[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const int k = 4 * s2 + lk;
      a1[s2] = W[k * kLD + bi * kNB + li];
      b1[s2] = Q1[k * kLD + bj * kNB + li];
      a2[s2] = Q1[k * kLD + bi * kNB + li];
      b2[s2] = W[k * kLD + bj * kNB + li];
    }
    const doublex4 m1 = mfma_k32(a1, b1);
    const bool diag = (P1 == P2);
    double off = 0.0, tot = 0.0, dmax = 0.0;
    const int col = bj * kNB + li;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int row = bi * kNB + lk + 4 * rr;
      const double v = m1[rr];
      store_through(&Anext[static_cast<int64_t>(gidx(I2, J2, row)) * N + gidx(I1, J1, col)], v);
      tot += v * v;
      if (diag && row == col) dmax = fmax(dmax, fabs(v));
      else off += v * v;
    }
    if (!diag) {
      const doublex4 m2 = mfma_k32(a2, b2);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        store_through(&Anext[static_cast<int64_t>(gidx(I1, J1, bi * kNB + lk + 4 * rr)) * N + gidx(I2, J2, col)],
                      m2[rr]);
      off *= 2.0;
      tot *= 2.0;
    }
    // fixed-order reduction: butterfly within each wave, then the 4 waves in order
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      off += __shfl_xor(off, m);
      tot += __shfl_xor(tot, m);
      dmax = fmax(dmax, __shfl_xor(dmax, m));
    }
    if (lane == 0) {
      red[3 * w + 0] = off;
      red[3 * w + 1] = tot;
      red[3 * w + 2] = dmax;
    }
    __syncthreads();
    if (t == 0 && tilepart) {  // null: a round whose norms nobody reads
      tilepart[3 * b + 0] = ((red[0] + red[3]) + red[6]) + red[9];
      tilepart[3 * b + 1] = ((red[1] + red[4]) + red[7]) + red[10];
      tilepart[3 * b + 2] = fmax(fmax(red[2], red[5]), fmax(red[8], red[11]));
    }
    return;
  }
  b -= ntiles;
  // ---- V piece: rows [32 rc, 32 rc + 32) of the columns of pair P, V <- V Q_P.
  // Computed as M = Q_P^T X^T (X = the piece) so that each wave's block is
  // stored by runs of consecutive rows; every wave has consumed its loads
  // before the barrier, after which the piece is overwritten in place.
  const int P = b % q, rc = b / q;
  int I, J;
  block_pair(p, r, P, I, J);
  const double* qg = Qcur + static_cast<int64_t>(P) * kS * kS;
  const int bm = w & 1, bn = w >> 1;
  double aq[8], bx[8];
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2) {
    const int k = 4 * s2 + lk;
    aq[s2] = qg[k + kS * (bm * kNB + li)];                                     // Q(k, j)
    bx[s2] = V[static_cast<int64_t>(gidx(I, J, k)) * N + rc * kS + bn * kNB + li];  // X(i, k)
  }
  const doublex4 acc = mfma_k32(aq, bx);
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
    store_through(&V[static_cast<int64_t>(gidx(I, J, bm * kNB + lk + 4 * rr)) * N + rc * kS + bn * kNB + li], acc[rr]);
}

__global__ void __launch_bounds__(256) k_jac_round(const double* __restrict__ Acur, double* __restrict__ Anext,
                                                   double* __restrict__ V, const double* __restrict__ Qcur,
                                                   double* __restrict__ Qnext, int N, int n, int r,
                                                   const double* __restrict__ scale, double* __restrict__ tilepart) {
  __shared__ double lds[kRoundLds];
  jac_round_body(blockIdx.x, Acur, Anext, V, Qcur, Qnext, N, n, r, scale, tilepart, lds);
}

// off-diagonal / total squared norms and max |diagonal| of A, per column
__device__ __forceinline__ void offnorm_cols_body(int c, const double* __restrict__ A, int N, int n,
                                                  double* __restrict__ part) {
  __shared__ double red[3][256];
  const int t = threadIdx.x;
  double off = 0.0, tot = 0.0;
  for (int rr = t; rr < n; rr += 256) {
    const double v = A[static_cast<int64_t>(c) * N + rr];
    tot += v * v;
    if (rr != c) off += v * v;
  }
  red[0][t] = off;
  red[1][t] = tot;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) {
      red[0][t] += red[0][t + s2];
      red[1][t] += red[1][t + s2];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[3 * c + 0] = red[0][0];
    part[3 * c + 1] = red[1][0];
    part[3 * c + 2] = fabs(A[static_cast<int64_t>(c) * N + c]);
  }
}

__global__ void __launch_bounds__(256) k_offnorm_cols(const double* __restrict__ A, int N, int n,
                                                      double* __restrict__ part) {
  offnorm_cols_body(blockIdx.x, A, N, n, part);
}

// reduce count (off, tot, dmax) triples in a fixed order: flags[0] = 1 if more
// sweeps are needed, flags[1] = 1 if non-finite, flags[2] = 1 if off(A) is
// small enough for a closing correction; scale[0] = max |a_ii|.
// flags is the device address of pinned host memory: the host reads it once
// the stream has drained, so the stores are system-scope (written through to
// host memory) and no copy is queued for them.
// (off, tot, dmax) over count partial triples, summed in a fixed order by the
// 256 threads of the workgroup; the totals are in red[.][0] afterwards
__device__ __forceinline__ void offnorm_reduce(const double* __restrict__ part, int count, double (*red)[256]) {
  const int t = threadIdx.x;
  double off = 0.0, tot = 0.0, dmax = 0.0;
  for (int c = t; c < count; c += 256) {
    off += part[3 * c];
    tot += part[3 * c + 1];
    dmax = fmax(dmax, part[3 * c + 2]);
  }
  red[0][t] = off;
  red[1][t] = tot;
  red[2][t] = dmax;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) {
      red[0][t] += red[0][t + s2];
      red[1][t] += red[1][t + s2];
      red[2][t] = fmax(red[2][t], red[2][t + s2]);
    }
    __syncthreads();
  }
}

// flags: more sweeps needed, non-finite, small enough for a closing correction
__device__ __forceinline__ void offnorm_flags(double off, double tot, int& more, int& nonfinite, int& small) {
  const bool finite = isfinite(tot);
  more = (finite && off > kOffTol * kOffTol * tot) ? 1 : 0;
  nonfinite = finite ? 0 : 1;
  small = (finite && off <= kCorrOff * kCorrOff * tot) ? 1 : 0;
}

// dctl (device memory, may be null): words 4 and 5 of a grouped solve's
// control block receive the first two flags as well
__device__ __forceinline__ void offnorm_final_body(const double* __restrict__ part, int count,
                                                   int* __restrict__ flags, double* __restrict__ scale,
                                                   int* __restrict__ dctl) {
  __shared__ double red[3][256];
  offnorm_reduce(part, count, red);
  if (threadIdx.x == 0) {
    int more, nonfinite, small;
    offnorm_flags(red[0][0], red[1][0], more, nonfinite, small);
    __hip_atomic_store(&flags[0], more, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&flags[1], nonfinite, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&flags[2], small, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    scale[0] = red[2][0];
    if (dctl) {
      dctl[4] = more;
      dctl[5] = nonfinite;
    }
  }
}

__global__ void __launch_bounds__(256) k_offnorm_final(const double* __restrict__ part, int count,
                                                       int* __restrict__ flags, double* __restrict__ scale,
                                                       int* __restrict__ dctl) {
  offnorm_final_body(part, count, flags, scale, dctl);
}

// Set-up of a solve, one pass over N x N: both A buffers cleared (their
// padded rows and columns must be zero; a solve that met non-finite values
// can leave NaN there) and V = [B_old 0; 0 I]: the rotations are accumulated
// straight into the previous eigenvectors, so the new ones need no final
// product B_old V
__device__ __forceinline__ void init_solve_body(int bx, double* __restrict__ V, double* __restrict__ A0,
                                                double* __restrict__ A1, int N, int n, const double* __restrict__ B,
                                                int ldb) {
  const int64_t i = static_cast<int64_t>(bx) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(N) * N) return;
  const int r = static_cast<int>(i % N), c = static_cast<int>(i / N);
  V[i] = (r < n && c < n) ? B[static_cast<int64_t>(c) * ldb + r] : (r == c ? 1.0 : 0.0);
  A0[i] = 0.0;
  A1[i] = 0.0;
}

__global__ void k_init_solve(double* __restrict__ V, double* __restrict__ A0, double* __restrict__ A1, int N, int n,
                             const double* __restrict__ B, int ldb) {
  init_solve_body(blockIdx.x, V, A0, A1, N, n, B, ldb);
}

// the set-up steps of the due descents of a grouped front (their warm start:
// kind GF_INIT clears A, A2 and sets V = B_old; the products are grouped
// dgemms; GF_OFFCOLS / GF_OFFFIN test the warm start as eigen_begin does)
__global__ void __launch_bounds__(256) kg_eigen_begin(int kind, const GFront* __restrict__ g,
                                                      const int* __restrict__ off, int count, GroupDueMask mask) {
  const int i = group_find(off, count, blockIdx.x);
  if (!due_mask_bit(mask, i)) return;
  const GFront& e = g[i];
  const int w = blockIdx.x - off[i];
  if (kind == GF_INIT)
    init_solve_body(w, e.V, e.A, e.A2, e.N, e.n, e.B, e.ldn);
  else if (kind == GF_OFFCOLS)
    offnorm_cols_body(w, e.A, e.N, e.n, e.epart);
  else
    offnorm_final_body(e.epart, e.n, e.dflags, e.scale, e.gctl);
}

// ---- closing correction.  Once the sweeps have made A nearly diagonal,
// rotating every index pair (i, j) at once by the angle that would
// annihilate a_ij in its own 2 x 2 subproblem,
//   theta_ij = atan(2 a_ij / (a_jj - a_ii)) / 2   (|theta_ij| <= pi/4),
// is a Newton-type step: the off-diagonal norm after it is of the order of
// its square over the relative eigenvalue gaps (Jacobi's method for
// symmetric matrices, quadratic convergence of simultaneous rotations).
// Theta is antisymmetric; the rotation Q = I + Theta + S/2 - S^2/8 with
// S = Theta^2 satisfies Q^T Q = I - S^3/8 + O(Theta^8), orthogonal to rounding
// for ||Theta||_F <= 2e-3, the acceptance bound.  A <- Q^T A Q and V <- V Q
// then take five float64 products instead of one more sweep's 63 rounds.

__global__ void k_diag(const double* __restrict__ A, int N, int n, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[static_cast<int64_t>(i) * N + i];
}

// Theta over 32 x 32 tiles: workgroup (bi >= bj) reads tiles (bi, bj) and
// (bj, bi) of A and writes both tiles of Theta and their sum of squares.
// A is symmetric only to rounding (the sweeps' diagonal tiles and the warm
// start are computed, not mirrored), and an angle magnifies that rounding by
// 1 / (a_jj - a_ii); so every angle is taken from (a_ij + a_ji) / 2, the
// same value for (i, j) and (j, i) because the sum commutes, which makes
// Theta antisymmetric bit for bit.  Entries at or below the sweeps' rotation
// threshold get no rotation, as in a sweep.
constexpr int kCT = 32;
__device__ __forceinline__ void lower_tile(int b, int& bi, int& bj) {
  bi = 0;
  while (b > bi) {  // lower tile index b -> (bi, bj), bj <= bi
    b -= bi + 1;
    ++bi;
  }
  bj = b;
}

__global__ void __launch_bounds__(256) k_corr_theta(const double* __restrict__ A, int N, int n,
                                                    const double* __restrict__ d, const double* __restrict__ scale,
                                                    double* __restrict__ Th, int ldt, double* __restrict__ part) {
  __shared__ double tl[kCT][kCT + 1], tu[kCT][kCT + 1];
  __shared__ double red[256];
  int bi, bj;
  lower_tile(blockIdx.x, bi, bj);
  const int t = threadIdx.x, tx = t & 31, ty = t >> 5;
  const int r0 = bi * kCT, c0 = bj * kCT;
  for (int k = ty; k < kCT; k += 8) {
    // tl[tx][k] = A(r0 + tx, c0 + k), tu[tx][k] = A(c0 + tx, r0 + k)
    tl[tx][k] = (r0 + tx < n && c0 + k < n) ? A[static_cast<int64_t>(c0 + k) * N + r0 + tx] : 0.0;
    tu[tx][k] = (c0 + tx < n && r0 + k < n) ? A[static_cast<int64_t>(r0 + k) * N + c0 + tx] : 0.0;
  }
  __syncthreads();
  const double thr = 2.2e-16 * scale[0];
  double acc = 0.0;
  for (int k = ty; k < kCT; k += 8) {
    const int r = r0 + tx, c = c0 + k;
    double th = 0.0;
    if (r < n && c < n && r != c) {
      const double a = 0.5 * (tl[tx][k] + tu[k][tx]);
      if (fabs(a) > thr) {
        const double g = r < c ? d[c] - d[r] : d[r] - d[c];  // d[max] - d[min]
        const double h = g < 0.0 ? 0.5 * atan2(-2.0 * a, -g) : 0.5 * atan2(2.0 * a, g);
        th = r < c ? h : -h;
      }
    }
    tl[tx][k] = th;  // each thread overwrites only the entries it read
    acc = fma(th, th, acc);
  }
  __syncthreads();
  for (int k = ty; k < kCT; k += 8) {
    if (r0 + tx < n && c0 + k < n) Th[static_cast<int64_t>(c0 + k) * ldt + r0 + tx] = tl[tx][k];
    // the mirror tile: Theta(c0 + tx, r0 + k) = -Theta(r0 + k, c0 + tx)
    if (bi != bj && c0 + tx < n && r0 + k < n) Th[static_cast<int64_t>(r0 + k) * ldt + c0 + tx] = -tl[k][tx];
  }
  red[t] = bi != bj ? 2.0 * acc : acc;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) red[t] += red[t + s2];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = red[0];
}

// Q = I + Theta + S/2 - S2/8 in place of Theta (rows, columns < n) if
// ||Theta||_F^2 = sum(part) <= theta2, else Q = I, which leaves A and V
// unchanged bit for bit.  Every workgroup reduces the count partial sums in the
// same order, so all take the same decision; workgroup 0 reports a rejection
// in flags[3] (pinned host memory, system-scope store).
__global__ void __launch_bounds__(256) k_corr_q(double* __restrict__ Th, int ldt, const double* __restrict__ S,
                                                int lds, const double* __restrict__ S2, int lds2, int n,
                                                const double* __restrict__ part, int count, double theta2,
                                                int* __restrict__ flags) {
  __shared__ double red[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double acc = 0.0;
  for (int i = t; i < count; i += 256) acc += part[i];
  red[t] = acc;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) red[t] += red[t + s2];
    __syncthreads();
  }
  const double tot = red[0];
  const bool accept = isfinite(tot) && tot <= theta2;
  if (c == 0 && t == 0) __hip_atomic_store(&flags[3], accept ? 0 : 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  for (int r = t; r < n; r += 256) {
    const int64_t i = static_cast<int64_t>(c) * ldt + r;
    double v = accept ? Th[i] + 0.5 * S[static_cast<int64_t>(c) * lds + r] -
                            0.125 * S2[static_cast<int64_t>(c) * lds2 + r]
                      : 0.0;
    if (r == c) v += 1.0;
    Th[i] = v;
  }
}

// dst = the lower triangle of src mirrored (n x n), 32 x 32 tiles through LDS:
// workgroup (bi >= bj) reads tile (bi, bj) and writes it and its transpose
__global__ void __launch_bounds__(256) k_sym_lower(const double* __restrict__ src, int lds, int n,
                                                   double* __restrict__ dst, int ldd) {
  __shared__ double tile[kCT][kCT + 1];
  int bi, bj;
  lower_tile(blockIdx.x, bi, bj);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int r0 = bi * kCT, c0 = bj * kCT;
  for (int k = ty; k < kCT; k += 8) {  // tile(row tx, col k)
    const int r = r0 + tx, c = c0 + k;
    tile[tx][k] = (r < n && c < n) ? src[static_cast<int64_t>(c) * lds + r] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < kCT; k += 8) {
    // (r0 + tx, c0 + k): lower of the tile, or its mirror on a diagonal tile
    const int r = r0 + tx, c = c0 + k;
    if (r < n && c < n) dst[static_cast<int64_t>(c) * ldd + r] = (bi == bj && tx < k) ? tile[k][tx] : tile[tx][k];
    // transpose: (c0 + tx, r0 + k) = tile(k, tx)
    const int r2 = c0 + tx, c2 = r0 + k;
    if (bi != bj && r2 < n && c2 < n) dst[static_cast<int64_t>(c2) * ldd + r2] = tile[k][tx];
  }
}

// dst[:n, :n] = src[:n, :n]
__global__ void k_copy_block(const double* __restrict__ src, int lds, int n, double* __restrict__ dst, int ldd) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r < n) dst[static_cast<int64_t>(c) * ldd + r] = src[static_cast<int64_t>(c) * lds + r];
}

// eigenvalue ranks (ascending, ties by index) and positive-definiteness flag;
// the diagonal is staged through LDS in chunks, kRankTPI threads count for one
// eigenvalue (every kRankTPI-th entry each) and sum their integer counts
constexpr int kRankTPI = 8;
__device__ __forceinline__ void eig_rank_body(int bx, const double* __restrict__ A, int N, int n,
                                              int32_t* __restrict__ perm, double* __restrict__ ev,
                                              const int* __restrict__ status, DevScalars* __restrict__ sc,
                                              double* dg) {
  const int sub = threadIdx.x % kRankTPI;
  const int i = bx * (256 / kRankTPI) + threadIdx.x / kRankTPI;
  const double vi = i < n ? A[static_cast<int64_t>(i) * N + i] : 0.0;
  int cnt = 0;
  for (int base = 0; base < n; base += 1024) {
    const int lim = min(1024, n - base);
    for (int j = threadIdx.x; j < lim; j += 256) dg[j] = A[static_cast<int64_t>(base + j) * N + base + j];
    __syncthreads();
#pragma unroll 8
    for (int j = sub; j < lim; j += kRankTPI) {
      const double vj = dg[j];
      cnt += (vj < vi) || (vj == vi && base + j < i);
    }
    __syncthreads();
  }
  // the kRankTPI counts of eigenvalue i sit in consecutive, aligned lanes
#pragma unroll
  for (int o = kRankTPI / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (i >= n || sub != 0) return;
  perm[cnt] = i;
  ev[i] = vi;
  if (cnt == 0) {
    sc->eig_ok = (vi > 0.0 && status[0] == 1) ? 1 : 0;
    sc->jac_sweeps = status[1];
    sc->jac_corr = status[2];
  }
}

__global__ void __launch_bounds__(256) k_eig_rank(const double* __restrict__ A, int N, int n,
                                                  int32_t* __restrict__ perm, double* __restrict__ ev,
                                                  const int* __restrict__ status, DevScalars* __restrict__ sc) {
  __shared__ double dg[1024];
  eig_rank_body(blockIdx.x, A, N, n, perm, ev, status, sc, dg);
}

// sign of each column: the entry of largest magnitude (first on ties) made positive
__device__ __forceinline__ void colsign_body(int c, const double* __restrict__ Bn, int ld, int n,
                                             double* __restrict__ sign, double* bv, int* bi) {
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

__global__ void __launch_bounds__(256) k_colsign(const double* __restrict__ Bn, int ld, int n,
                                                 double* __restrict__ sign) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  colsign_body(blockIdx.x, Bn, ld, n, sign, bv, bi);
}

template <typename T>
__device__ __forceinline__ void permute_body(int bx, int r, const double* __restrict__ Bn, int ldt, int n,
                                             const int32_t* __restrict__ perm, const double* __restrict__ ev,
                                             const double* __restrict__ sign, double* __restrict__ B, int ldb,
                                             double* __restrict__ D, T* __restrict__ BD, int ldbd) {
  const int row = bx * blockDim.x + threadIdx.x;  // r: output column
  const int c = perm[r];
  const double d = sqrt(fmax(ev[c], 0.0));
  if (row == 0) D[r] = d;
  if (row >= n) return;
  const double v = sign[c] * Bn[static_cast<int64_t>(c) * ldt + row];
  B[static_cast<int64_t>(r) * ldb + row] = v;
  BD[static_cast<int64_t>(r) * ldbd + row] = static_cast<T>(v * d);
}

template <typename T>
__global__ void __launch_bounds__(256) k_permute(const double* __restrict__ Bn, int ldt, int n,
                                                 const int32_t* __restrict__ perm, const double* __restrict__ ev,
                                                 const double* __restrict__ sign, double* __restrict__ B, int ldb,
                                                 double* __restrict__ D, T* __restrict__ BD, int ldbd) {
  permute_body<T>(blockIdx.x, blockIdx.y, Bn, ldt, n, perm, ev, sign, B, ldb, D, BD, ldbd);
}

// ---- grouped eigensolve: the sweeps of many descents (one per entry of a
// descriptor table, uneven n allowed) advance together, one launch per round
// for all of them.  Each launch's workgroups are split over the descents by a
// prefix-sum table (workgroup w belongs to descent i with off[i] <= w <
// off[i + 1]); a descent's convergence is decided on the device, after each
// of its sweeps, at the start of the next round (see kg_round), so the host
// only waits for the whole group.
// The arithmetic of every step is that of the single-descent solve (the same
// bodies, the same reduction order), without the closing correction.

__device__ __forceinline__ bool due_bit(const GroupDueMask& m, int i) { return (m.w[i >> 5] >> (i & 31)) & 1u; }

// whether each descent's solve sweeps at all (from the warm start's flags and
// the previous solve's sweep count, as the single-descent solve decides), and
// the control words of the solve; one workgroup, a thread per descent.  The
// number of sweeping descents goes to the device counter dactive and, in one
// system-scope store, to the host's copy (per-descent atomics on host memory
// would each make a round trip over the bus, one after another).
__global__ void __launch_bounds__(256) kg_start(const GEigDesc* __restrict__ g, int count, GroupDueMask due,
                                                int max_sweeps, int* __restrict__ dactive,
                                                int* __restrict__ hactive, int* __restrict__ hsweeps) {
  __shared__ int cnt[256];
  int act = 0;
  for (int i = threadIdx.x; i < count; i += 256) {
    if (g[i].N == kS) continue;  // N = 32: kg_small_solve
    int* c = g[i].ctl;
    const int d = due_bit(due, i) ? 1 : 0;
    c[GC_DUE] = d;
    if (!d) continue;
    const int last = c[GC_LAST];
    const int mins = last >= 2 ? min(last - 1, max_sweeps) : 0;
    const int more = c[GC_MORE], nonfin = c[GC_NONFIN];
    const bool active = mins > 0 || (more && !nonfin);
    c[GC_MIN] = mins;
    if (active) {
      c[GC_STOPR] = 0x7fffffff;
      ++act;
    } else {
      c[GC_STOPR] = 0;
      c[GC_LAST] = 0;
      int* st = g[i].status;
      st[0] = nonfin ? 3 : (more ? 2 : 1);
      st[1] = 0;
      st[2] = 0;
      __hip_atomic_store(&hsweeps[i], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&hsweeps[kGroupMax + i], st[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  cnt[threadIdx.x] = act;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) cnt[threadIdx.x] += cnt[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __hip_atomic_store(dactive, cnt[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(hactive, cnt[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// the first pair solves (round 0 with the intra-block rotations) of every
// sweeping descent, from its warm-started A
__global__ void __launch_bounds__(256) kg_first(const GEigDesc* __restrict__ g, const int* __restrict__ off,
                                                int count) {
  __shared__ double lds[3 * kS * kLD];
  const int i = group_find(off, count, blockIdx.x);
  const GEigDesc& e = g[i];
  if (!e.ctl[GC_DUE] || e.ctl[GC_STOPR] == 0) return;
  jac_first_body(blockIdx.x - off[i], e.A, e.N, e.n, e.N / kNB, e.scale, e.Q, lds);
}

// global round rg of the group: descent i runs its round rg mod (p_i - 1)
// (every descent starts its first sweep at rg = 0) until the round after the
// one in which it stopped; A and Q ping-pong with the parity of rg.  The
// scale that sets the rotation threshold is double buffered by sweep parity:
// sweep s reads scale[s & 1], written when sweep s - 1 is decided.
// The launch puts every descent's pair solves first (offq: prefix sums of
// the q_i), then the tile and V workgroups (off: prefix sums of whole rounds,
// so off[i] - offq[i] is descent i's first tile-or-V workgroup): the pair
// solves, the round's critical path, are then dispatched ahead of the rest
// and spread over distinct CUs instead of sharing some CUs two by two.
// uq > 0: every descent of the group has the same q = uq and uq + ur tile
// and V workgroups, so the slot follows by division (no search).
__device__ __forceinline__ void round_slot(const int* __restrict__ offq, const int* __restrict__ off, int count,
                                           int uq, int ur, int w, int& i, int& b) {
  if (uq > 0) {
    const int tq = uq * count;
    if (w < tq) {
      i = w / uq;
      b = w - i * uq;
    } else {
      w -= tq;
      i = w / ur;
      b = uq + (w - i * ur);
    }
    return;
  }
  const int tq = offq[count];
  if (w < tq) {
    i = group_find(offq, count, w);
    b = w - offq[i];
    return;
  }
  w -= tq;
  int lo = 0, hi = count;  // the last i with off[i] - offq[i] <= w
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] - offq[mid] <= w) lo = mid;
    else hi = mid;
  }
  i = lo;
  b = (offq[i + 1] - offq[i]) + (w - (off[i] - offq[i]));
}

// The decision on sweep s (more sweeps, the next rotation threshold) is
// taken at the start of the next launch, the first round of sweep s + 1, by
// every workgroup of the descent alike: each sums the partial norms of sweep
// s's last round in the same fixed order, so all reach the same decision
// without waiting for one another; workgroup 0 records it.  Only that last
// round writes the partial sums.  (Deciding inside the last round instead
// needs a device-wide fence in every tile workgroup, an L2 write-back and
// invalidate each, which slowed the pair solves running beside them; a
// launch of its own between the rounds costs a dependent launch per sweep.)
__global__ void __launch_bounds__(256) kg_round(const GEigDesc* __restrict__ g, const int* __restrict__ offq,
                                                const int* __restrict__ off, int count, int uq, int ur, int rg,
                                                int max_sweeps,
                                                int* __restrict__ dactive, int* __restrict__ hactive,
                                                int* __restrict__ hsweeps) {
  __shared__ double lds[kRoundLds];
  __shared__ double red[3][256];
  int i, b;
  round_slot(offq, off, count, uq, ur, blockIdx.x, i, b);
  const GEigDesc& e = g[i];
  int* c = e.ctl;
  if (!c[GC_DUE] || rg >= c[GC_STOPR]) return;
  const int N = e.N, p = N / kNB, q = p / 2, ntiles = q * (q + 1) / 2;
  const int rl = rg % (p - 1), sw = rg / (p - 1);
  const bool odd = rg & 1;
  const double* scale = e.scale + (sw & 1);
  if (rl == 0 && sw > 0) {
    offnorm_reduce(e.part, ntiles, red);
    int more, nonfin, small;
    offnorm_flags(red[0][0], red[1][0], more, nonfin, small);
    const int done = sw;
    const bool cont = done < max_sweeps && (done < c[GC_MIN] || (more && !nonfin));
    if (b == 0 && threadIdx.x == 0) {
      if (cont) {
        e.scale[sw & 1] = red[2][0];
      } else {
        c[GC_STOPR] = rg;
        c[GC_LAST] = done;
        int* st = e.status;
        st[0] = nonfin ? 3 : (more ? 2 : 1);
        st[1] = done;
        st[2] = 0;
        __hip_atomic_store(&hsweeps[i], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&hsweeps[kGroupMax + i], st[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        // the descent that stops last tells the host (one store over the bus)
        if (__hip_atomic_fetch_add(dactive, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1)
          __hip_atomic_store(hactive, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    if (!cont) return;
    scale = &red[2][0];  // this launch's pair solves use the new threshold at once
  }
  jac_round_body(b, odd ? e.A2 : e.A, odd ? e.A : e.A2, e.V, odd ? e.Q2 : e.Q, odd ? e.Q : e.Q2, N, e.n, rl, scale,
                 rl == p - 2 ? e.part : nullptr, lds);
}

// ---- whole solve of a descent with N = 32 (n <= 32) in one workgroup, from
// the warm start to the canonical B, D and B D.  The warm start A = B_old^T C
// B_old and V = B_old are formed in LDS, and whether to sweep at all is decided
// from A's off-diagonal norm and the previous solve's sweep count as kg_start
// decides it.  With two blocks there is a single block pair, so a sweep is one
// pair solve on the whole matrix: the rotations of rotate_pair (intra-block
// rounds, then cross rounds) give Q, then A <- Q^T A Q and V <- V Q are formed
// on the float64 matrix cores, and the off-diagonal norm decides on the next
// sweep, all inside the kernel.  The stopping rule, the rotation threshold
// (from the previous max |a_ii|) and the sweep accounting are those of
// kg_round; the finishing steps (ranks, column signs, canonical B, D and B D)
// follow in the same workgroup.  Later launches of a mixed group skip the
// descent (kg_start leaves it alone, its due word is cleared).

// P = X Y for 32 x 32 matrices in LDS (row stride kLD), X given as X(r, k) =
// xs[r * kLD + k] or, with XT, as xs[k * kLD + r]; each of the four waves
// forms one 16 x 16 block of P (mfma_k32 layout)
template <bool XT>
__device__ __forceinline__ doublex4 small_product(const double* xs, const double* ys, int bi, int bj) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  double a[8], b[8];
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2) {
    const int k = 4 * s2 + lk;
    a[s2] = XT ? xs[k * kLD + bi * kNB + li] : xs[(bi * kNB + li) * kLD + k];
    b[s2] = ys[k * kLD + bj * kNB + li];
  }
  return mfma_k32(a, b);
}

// off-diagonal / total squared norms over the n x n part of Aw and max
// |a_ii|: one column per thread, then the columns in order by thread 0, which
// gets the flags (as offnorm_flags) and the new scale in red[2][0]
__device__ __forceinline__ void small_offnorm(const double* Aw, int n, double (*red)[kS], int& more, int& nonfin) {
  const int t = threadIdx.x;
  if (t < kS) {
    double off = 0.0, tot = 0.0;
    for (int r = 0; r < n; ++r) {
      const double v = Aw[r * kLD + t];
      tot += v * v;
      if (r != t) off += v * v;
    }
    red[0][t] = t < n ? off : 0.0;
    red[1][t] = t < n ? tot : 0.0;
    red[2][t] = t < n ? fabs(Aw[t * kLD + t]) : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    double off = 0.0, tot = 0.0, dmax = 0.0;
    for (int k = 0; k < kS; ++k) {
      off += red[0][k];
      tot += red[1][k];
      dmax = fmax(dmax, red[2][k]);
    }
    red[2][0] = dmax;
    int small;
    offnorm_flags(off, tot, more, nonfin, small);
  }
}

__global__ void __launch_bounds__(256) kg_small_solve(const GEigDesc* __restrict__ g, int count, GroupDueMask due,
                                                      int max_sweeps, int* __restrict__ hsweeps) {
  __shared__ double Aw[kS * kLD], S0[kS * kLD], S1[kS * kLD], Q[kS * kLD], Vw[kS * kLD], T[kS * kLD];
  __shared__ double red[3][kS];
  __shared__ double ev[kS], sgn[kS];
  __shared__ int perm[kS];
  __shared__ int go;
  const int i = blockIdx.x;
  if (i >= count) return;
  const GEigDesc& e = g[i];
  if (e.N != kS) return;
  int* c = e.ctl;
  const int n = e.n, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4, bi = w & 1, bj = w >> 1;
  if (!due_mask_bit(due, i)) {
    if (t == 0) c[GC_DUE] = 0;
    return;
  }
  // warm start: C and V = B_old padded with zeros / the identity; T = C V,
  // then A = V^T T (mirrored from its lower half)
  for (int idx = t; idx < kS * kS; idx += 256) {
    const int r = idx % kS, cc = idx / kS;
    const bool in = r < n && cc < n;
    S0[r * kLD + cc] = in ? e.C[static_cast<int64_t>(cc) * e.ldc + r] : 0.0;
    Vw[r * kLD + cc] = in ? e.B[static_cast<int64_t>(cc) * e.ldb + r] : (r == cc ? 1.0 : 0.0);
  }
  __syncthreads();
  {
    const doublex4 cv = small_product<false>(S0, Vw, bi, bj);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) T[(bi * kNB + lk + 4 * rr) * kLD + bj * kNB + li] = cv[rr];
    __syncthreads();
    const doublex4 vt = small_product<true>(Vw, T, bi, bj);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) Aw[(bi * kNB + lk + 4 * rr) * kLD + bj * kNB + li] = vt[rr];
    __syncthreads();
    for (int idx = t; idx < kS * kS; idx += 256) {
      const int r = idx / kS, cc = idx % kS;
      if (r < cc) Aw[r * kLD + cc] = Aw[cc * kLD + r];
    }
    __syncthreads();
  }
  int done = 0, more = 0, nonfin = 0;
  small_offnorm(Aw, n, red, more, nonfin);
  // whether to sweep (kg_start): at least last - 1 sweeps after a solve of
  // `last` sweeps, else only while the warm start is not diagonal enough
  const int last = c[GC_LAST];
  const int mins = last >= 2 ? min(last - 1, max_sweeps) : 0;
  if (t == 0) go = (mins > 0 || (more && !nonfin)) ? 1 : 0;
  __syncthreads();
  const bool active = go != 0;
  double scale = red[2][0];
  __syncthreads();
  while (active) {
    for (int idx = t; idx < kS * kS; idx += 256) S0[(idx / kS) * kLD + idx % kS] = Aw[(idx / kS) * kLD + idx % kS];
    __syncthreads();
    rotate_pair(S0, S1, Q, 2.2e-16 * scale, scale > 0.0 ? 1.0 / scale : 0.0, true, nullptr, false, kNB >= n);
    // T = A Q and V Q (into S1), then A = Q^T T, mirrored from its lower half
    const doublex4 aq = small_product<false>(Aw, Q, bi, bj);
    const doublex4 vq = small_product<false>(Vw, Q, bi, bj);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      T[(bi * kNB + lk + 4 * rr) * kLD + bj * kNB + li] = aq[rr];
      S1[(bi * kNB + lk + 4 * rr) * kLD + bj * kNB + li] = vq[rr];
    }
    __syncthreads();
    const doublex4 qt = small_product<true>(Q, T, bi, bj);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) Aw[(bi * kNB + lk + 4 * rr) * kLD + bj * kNB + li] = qt[rr];
    __syncthreads();
    for (int idx = t; idx < kS * kS; idx += 256) {
      const int r = idx / kS, cc = idx % kS;
      if (r < cc) Aw[r * kLD + cc] = Aw[cc * kLD + r];
      Vw[r * kLD + cc] = S1[r * kLD + cc];
    }
    __syncthreads();
    small_offnorm(Aw, n, red, more, nonfin);
    if (t == 0) {
      ++done;
      go = (done < max_sweeps && (done < mins || (more && !nonfin))) ? 1 : 0;
    }
    __syncthreads();
    scale = red[2][0];
    if (!go) break;
    __syncthreads();
  }
  if (t == 0) {
    int* st = e.status;
    st[0] = nonfin ? 3 : (more ? 2 : 1);
    st[1] = done;
    st[2] = 0;
    c[GC_LAST] = done;
    c[GC_STOPR] = 0;
    c[GC_DUE] = 0;
    __hip_atomic_store(&hsweeps[i], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&hsweeps[kGroupMax + i], st[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  // finishing steps, as kg_rank / kg_colsign / kg_permute: ascending
  // eigenvalues (ties by index), each column's largest-magnitude entry (first
  // on ties) positive, then B, D and B D in that order
  if (t < kS) {
    ev[t] = Aw[t * kLD + t];
    perm[t] = t;  // (non-finite eigenvalues can leave ranks unassigned)
  }
  __syncthreads();
  if (t < n) {
    const double vi = ev[t];
    int cnt = 0;
    for (int j = 0; j < n; ++j) cnt += (ev[j] < vi) || (ev[j] == vi && j < t);
    perm[cnt] = t;
    e.perm[cnt] = t;
    e.evals[t] = vi;
    double best = -1.0;
    int arg = 0;
    for (int r = 0; r < n; ++r) {
      const double v = fabs(Vw[r * kLD + t]);
      if (v > best) {
        best = v;
        arg = r;
      }
    }
    sgn[t] = Vw[arg * kLD + t] < 0.0 ? -1.0 : 1.0;
    e.sign[t] = sgn[t];
    if (cnt == 0) {
      const int* st = e.status;
      e.sc->eig_ok = (vi > 0.0 && st[0] == 1) ? 1 : 0;
      e.sc->jac_sweeps = st[1];
      e.sc->jac_corr = st[2];
    }
  }
  __syncthreads();
  for (int idx = t; idx < n * n; idx += 256) {
    const int r = idx / n, row = idx % n;  // output column r, row
    const int cc = min(max(perm[r], 0), n - 1);
    const double d = sqrt(fmax(ev[cc], 0.0));
    const double v = sgn[cc] * Vw[row * kLD + cc];
    if (row == 0) e.D[r] = d;
    e.B[static_cast<int64_t>(r) * e.ldb + row] = v;
    if (e.bd64)
      static_cast<double*>(e.BD)[static_cast<int64_t>(r) * e.ldbd + row] = v * d;
    else
      static_cast<float*>(e.BD)[static_cast<int64_t>(r) * e.ldbd + row] = static_cast<float>(v * d);
  }
}

// the finishing steps of every descent that solved: eigenvalue ranks, column
// signs, then the canonical B, D and B D (A and V as left by its last round)
__global__ void __launch_bounds__(256) kg_rank(const GEigDesc* __restrict__ g, const int* __restrict__ off,
                                               int count) {
  __shared__ double dg[1024];
  const int i = group_find(off, count, blockIdx.x);
  const GEigDesc& e = g[i];
  if (!e.ctl[GC_DUE]) return;
  const double* A = (e.status[1] & 1) ? e.A2 : e.A;
  eig_rank_body(blockIdx.x - off[i], A, e.N, e.n, e.perm, e.evals, e.status, e.sc, dg);
}

__global__ void __launch_bounds__(256) kg_colsign(const GEigDesc* __restrict__ g, const int* __restrict__ off,
                                                  int count) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int i = group_find(off, count, blockIdx.x);
  const GEigDesc& e = g[i];
  if (!e.ctl[GC_DUE]) return;
  colsign_body(blockIdx.x - off[i], e.V, e.N, e.n, e.sign, bv, bi);
}

__global__ void __launch_bounds__(256) kg_permute(const GEigDesc* __restrict__ g, const int* __restrict__ off,
                                                  int count) {
  const int i = group_find(off, count, blockIdx.x);
  const GEigDesc& e = g[i];
  if (!e.ctl[GC_DUE]) return;
  const int nb = (e.n + 255) / 256, w = blockIdx.x - off[i];
  if (e.bd64)
    permute_body<double>(w % nb, w / nb, e.V, e.N, e.n, e.perm, e.evals, e.sign, e.B, e.ldb, e.D,
                         static_cast<double*>(e.BD), e.ldbd);
  else
    permute_body<float>(w % nb, w / nb, e.V, e.N, e.n, e.perm, e.evals, e.sign, e.B, e.ldb, e.D,
                        static_cast<float*>(e.BD), e.ldbd);
}

}  // namespace

// ---- host side: the eigensolve as a resumable sequence, so several
// descents can advance their sweeps in lockstep with one host
// synchronisation per sweep (the convergence flag is the only value the
// host needs between sweeps; it lands in pinned host memory).

void eigen_begin_host(EigWork& w) {
  w.Acur = w.A;
  w.Anext = w.A2;
  w.Qcur = w.Q;
  w.Qnext = w.Q2;
  w.sweeps = 0;
  w.corrections = 0;
  w.fresh = true;
  w.corr_queued = false;
  w.corr_blocked = false;
  w.pending = true;
}

int eigen_begin(hipStream_t st, int n, const double* C, int ldc, const double* B, int ldb, EigWork& w,
                KTimer* kt) {
  const int N = w.N;
  const int64_t NN = static_cast<int64_t>(N) * N;
  eigen_begin_host(w);
  k_init_solve<<<static_cast<int>((NN + 255) / 256), 256, 0, st>>>(w.V, w.Acur, w.Anext, N, n, B, ldb);
  CMX_HIP(hipGetLastError());
  kt_begin(kt, KID_EIG_GEMM);
  CMX_HIP(launch_dgemm_ksplit(st, false, false, n, n, n, C, ldc, B, ldb, w.T, ldb, w.X2, N));   // T = C B
  kt_end(kt);
  kt_begin(kt, KID_EIG_GEMM);
  CMX_HIP(launch_dgemm_ksplit(st, true, false, n, n, n, B, ldb, w.T, ldb, w.Acur, N, w.X2, N));   // A = B^T T
  kt_end(kt);
  k_offnorm_cols<<<n, 256, 0, st>>>(w.Acur, N, n, w.part);
  k_offnorm_final<<<1, 256, 0, st>>>(w.part, n, w.dflags, w.scale, w.gctl);
  CMX_HIP(hipGetLastError());
  w.pending = true;
  return 0;
}

__global__ void k_set_status(int* status, int code, int sweeps, int corrections) {
  if (threadIdx.x == 0) {
    status[0] = code;
    status[1] = sweeps;
    status[2] = corrections;
  }
}

void eigen_drop_graphs(EigWork& w) {
  for (auto& g : w.gx) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  w.gstream = nullptr;
}

int eigen_step(hipStream_t st, int n, double* B, int ldb, double* D, void* BD, bool fp64_bd, int ldbd, EigWork& w,
               DevScalars* sc, int max_sweeps, KTimer* kt, bool use_graph, bool* done, bool ahead) {
  *done = false;
  const int N = w.N;
  const int p = N / kNB, q = p / 2;
  const int ntiles = q * (q + 1) / 2;
  // ahead: the first batch of a warm-started solve, queued behind the warm
  // start before its flags are read (a solve after one that took several
  // sweeps needs at least that batch; on a converged or non-finite warm
  // start the extra sweeps change nothing that the next check does not see)
  if (ahead && (w.sweeps != 0 || w.last_sweeps < 2)) return 0;
  if (!ahead && w.corr_queued) {  // a rejected correction (its rotation was not small) is not tried again
    if (w.hflags[3] || w.corrections >= kMaxCorrections) w.corr_blocked = true;
    w.corr_queued = false;
  }
  const bool more = ahead || (w.hflags[0] && !w.hflags[1]);
  if (more && w.sweeps < max_sweeps) {
    const int round_blocks = q + ntiles + (N / kS) * q;
    // one sweep's launches (sweeps alternate between the two A and Q buffers
    // because a sweep has an odd number p - 1 of rounds)
    auto queue_sweep = [&](double* a0, double* a1, double* q0, double* q1, bool first) -> hipError_t {
      if (first) {
        kt_begin(kt, KID_JACOBI);
        k_jac_first<<<q, 256, 0, st>>>(a0, N, n, p, w.scale, q0);
        kt_end(kt);
      }
      for (int r = 0; r < p - 1; ++r) {
        hipEvent_t t0, t1;
        if (kt_ext(kt, KID_JACOBI, &t0, &t1))
          hipExtLaunchKernelGGL(k_jac_round, dim3(round_blocks), dim3(256), 0, st, t0, t1, 0, a0, a1, w.V, q0, q1,
                                N, n, r, w.scale, w.part);
        else
          k_jac_round<<<round_blocks, 256, 0, st>>>(a0, a1, w.V, q0, q1, N, n, r, w.scale, w.part);
        std::swap(a0, a1);
        std::swap(q0, q1);
      }
      k_offnorm_final<<<1, 256, 0, st>>>(w.part, ntiles, w.dflags, w.scale, nullptr);
      return hipGetLastError();
    };
    // one closing correction from a0 into a1 (X1: Theta, then Q; X2: S, then
    // A Q; a1: S^2, then V Q, then the result; the k-split products use a1 or
    // T as scratch while those are free)
    auto queue_correction = [&](double* a0, double* a1) -> hipError_t {
      hipError_t e;
      k_diag<<<ceil_div(n, 256), 256, 0, st>>>(a0, N, n, w.evals);
      const int nt = ceil_div(n, kCT), ntl = nt * (nt + 1) / 2;
      k_corr_theta<<<ntl, 256, 0, st>>>(a0, N, n, w.evals, w.scale, w.X1, N, w.part);
      kt_begin(kt, KID_EIG_GEMM);
      e = launch_dgemm_ksplit(st, false, false, n, n, n, w.X1, N, w.X1, N, w.X2, N, a1, N);  // S = Theta^2
      kt_end(kt);
      if (e != hipSuccess) return e;
      kt_begin(kt, KID_EIG_GEMM);
      e = launch_dgemm_ksplit(st, false, false, n, n, n, w.X2, N, w.X2, N, a1, N, w.T, ldb);  // S^2
      kt_end(kt);
      if (e != hipSuccess) return e;
      k_corr_q<<<n, 256, 0, st>>>(w.X1, N, w.X2, N, a1, N, n, w.part, ntl, w.corr_max_theta * w.corr_max_theta,
                                  w.dflags);
      kt_begin(kt, KID_EIG_GEMM);
      e = launch_dgemm2(st, n, n, n, a0, N, w.V, N, w.X1, N, w.X2, N, a1, N);  // A Q and V Q
      kt_end(kt);
      if (e != hipSuccess) return e;
      k_copy_block<<<dim3(ceil_div(n, 256), n), 256, 0, st>>>(a1, N, n, w.V, N);
      kt_begin(kt, KID_EIG_GEMM);
      e = launch_dgemm_ksplit(st, true, false, n, n, n, w.X1, N, w.X2, N, w.T, ldb, a1, N);  // Q^T (A Q)
      kt_end(kt);
      if (e != hipSuccess) return e;
      k_sym_lower<<<ntl, 256, 0, st>>>(w.T, ldb, n, a1, N);
      k_offnorm_cols<<<n, 256, 0, st>>>(a1, N, n, w.part);
      k_offnorm_final<<<1, 256, 0, st>>>(w.part, n, w.dflags, w.scale, nullptr);
      return hipGetLastError();
    };
    // replay step `slot` from a graph captured on first use (queue() queues
    // its launches), or queue it directly
    auto run = [&](int slot, const std::function<hipError_t()>& queue) -> int {
      if (!(use_graph && !(kt && kt->on))) {
        CMX_HIP(queue());
        return 0;
      }
      if (w.gx[slot] == nullptr || w.gstream != st) {
        if (w.gstream != st) eigen_drop_graphs(w);
        CMX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const hipError_t qe = queue();
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(st, &g);
        if (qe != hipSuccess || ce != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return fail(-3, std::string("eigen step capture: ") + hipGetErrorString(qe != hipSuccess ? qe : ce));
        }
        const hipError_t ie = hipGraphInstantiate(&w.gx[slot], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(-3, std::string("eigen step graph: ") + hipGetErrorString(ie));
        w.gstream = st;
      }
      CMX_HIP(hipGraphLaunch(w.gx[slot], st));
      return 0;
    };
    const bool from_a = (w.Acur == w.A);
    if (!ahead && w.correct_on && !w.corr_blocked && w.hflags[2]) {
      double *a0 = w.Acur, *a1 = w.Anext;
      if (const int rc = run(from_a ? 4 : 5, [&] { return queue_correction(a0, a1); })) return rc;
      // the Q buffers flip with the A buffers, as in a round: the captured
      // sweeps are keyed by the A buffer they start from and assume the
      // matching Q buffer (the next sweep recomputes its first pair
      // solves from A, so the Q contents do not matter)
      std::swap(w.Acur, w.Anext);
      std::swap(w.Qcur, w.Qnext);
      ++w.sweeps;
      ++w.corrections;
      w.fresh = true;  // the pair solves the last sweep carried over are stale
      w.corr_queued = true;
      return 0;
    }
    // the first check queues as many sweeps as the previous solve ran before
    // its closing correction (one fewer if it closed with a sweep): a
    // warm-started solve rarely needs fewer, and while it needs at least as
    // many the sweeps run are those of a check after every sweep
    int batch = 1;
    if (w.sweeps == 0) batch = std::max(1, w.last_closed ? w.last_sweeps : w.last_sweeps - 1);
    batch = std::min(batch, max_sweeps - w.sweeps);
    for (int i = 0; i < batch; ++i) {
      const bool first = w.fresh;
      const int slot = first ? (w.Acur == w.A ? 2 : 3) : (w.Acur == w.A ? 0 : 1);
      double *a0 = w.Acur, *a1 = w.Anext, *q0 = w.Qcur, *q1 = w.Qnext;
      if (const int rc = run(slot, [&] { return queue_sweep(a0, a1, q0, q1, first); })) return rc;
      for (int r = 0; r < p - 1; ++r) {
        std::swap(w.Acur, w.Anext);
        std::swap(w.Qcur, w.Qnext);
      }
      ++w.sweeps;
      w.fresh = false;
    }
    return 0;
  }
  // converged (1), sweep limit (2) or non-finite (3): finish
  k_set_status<<<1, 64, 0, st>>>(w.status, w.hflags[1] ? 3 : (w.hflags[0] ? 2 : 1), w.sweeps - w.corrections,
                                 w.corrections);
  // V holds B_new = B_old V_rot: canonical order / signs into B, D, BD
  k_eig_rank<<<ceil_div(n, 256 / kRankTPI), 256, 0, st>>>(w.Acur, N, n, w.perm, w.evals, w.status, sc);
  k_colsign<<<n, 256, 0, st>>>(w.V, N, n, w.sign);
  dim3 grid(ceil_div(n, 256), n);
  if (fp64_bd)
    k_permute<double><<<grid, 256, 0, st>>>(w.V, N, n, w.perm, w.evals, w.sign, B, ldb, D,
                                            static_cast<double*>(BD), ldbd);
  else
    k_permute<float><<<grid, 256, 0, st>>>(w.V, N, n, w.perm, w.evals, w.sign, B, ldb, D,
                                           static_cast<float*>(BD), ldbd);
  CMX_HIP(hipGetLastError());
  w.pending = false;
  w.last_sweeps = w.sweeps - w.corrections;
  w.last_closed = w.corrections > 0;
  *done = true;
  return 0;
}


hipError_t launch_group_eigen_begin(hipStream_t st, int kind, const GFront* g, const int* off, int count, int wgs,
                                    const GroupDueMask& mask) {
  if (wgs > 0) kg_eigen_begin<<<wgs, 256, 0, st>>>(kind, g, off, count, mask);
  return hipGetLastError();
}

// ---- host side of the grouped eigensolve

void group_eig_release(GroupEig& ge) {
  if (ge.dtab) (void)hipFree(ge.dtab);
  if (ge.hflags) (void)hipHostFree(ge.hflags);
  ge = GroupEig{};
}

int group_eig_build(hipStream_t st, GroupEig& ge, const std::vector<GEigDesc>& descs) {
  const int count = static_cast<int>(descs.size());
  if (count < 1 || count > kGroupMax) return fail(-1, "grouped eigensolve: 1 to 1024 descents");
  // workgroups per descent of each kind: first, round, rank, colsign, permute
  std::vector<int> off(kGroupKinds * (count + 1), 0);
  for (int i = 0; i < count; ++i) {
    const GEigDesc& e = descs[i];
    const int N = e.N, p = N / kNB, q = p / 2, ntiles = q * (q + 1) / 2;
    const int wgs[kGroupKinds] = {q, q + ntiles + (N / kS) * q, ceil_div(e.n, 256 / kRankTPI), e.n,
                                  ceil_div(e.n, 256) * e.n};
    for (int k = 0; k < kGroupKinds; ++k) off[k * (count + 1) + i + 1] = off[k * (count + 1) + i] + wgs[k];
  }
  int pmax = 2, nsmall = 0;
  bool uniform = true;  // every descent has the same padded size
  for (const auto& e : descs) {
    pmax = std::max(pmax, e.N / kNB);
    nsmall += e.N == kS ? 1 : 0;
    uniform = uniform && e.N == descs[0].N;
  }
  const size_t tab_bytes = sizeof(GEigDesc) * count, off_bytes = sizeof(int) * off.size();
  if (ge.cap < count) {
    group_eig_release(ge);
    void* d = nullptr;
    const size_t tab_off = sizeof(GEigDesc) * kGroupMax + sizeof(int) * kGroupKinds * (kGroupMax + 1);
    const size_t cnt_off = (tab_off + 255) / 256 * 256;  // the device count of sweeping descents
    if (hipMalloc(&d, cnt_off + 256) != hipSuccess) return fail(-2, "grouped eigensolve: hipMalloc failed");
    ge.dtab = d;
    ge.dactive = reinterpret_cast<int*>(static_cast<char*>(d) + cnt_off);
    void* hf = nullptr;
    if (hipHostMalloc(&hf, sizeof(int) * (2 * kGroupMax + 1), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
      return fail(-2, "grouped eigensolve: hipHostMalloc failed");
    ge.hflags = static_cast<int*>(hf);
    void* dp = nullptr;
    CMX_HIP(hipHostGetDevicePointer(&dp, hf, 0));
    ge.dflags = static_cast<int*>(dp);
    ge.cap = kGroupMax;
  }
  ge.count = count;
  ge.pmax = pmax;
  ge.nsmall = nsmall;
  {
    const int q = descs[0].N / kNB / 2;
    ge.uq = uniform ? q : 0;
    ge.ur = uniform ? off[1 * (count + 1) + 1] - q : 0;  // tile and V workgroups of one descent
  }
  ge.off = off;
  // the table and the offsets, on the group's stream; consumed before return
  CMX_HIP(hipMemcpyAsync(ge.dtab, descs.data(), tab_bytes, hipMemcpyHostToDevice, st));
  CMX_HIP(hipMemcpyAsync(static_cast<char*>(ge.dtab) + sizeof(GEigDesc) * kGroupMax, off.data(), off_bytes,
                         hipMemcpyHostToDevice, st));
  CMX_HIP(hipStreamSynchronize(st));
  return 0;
}

int group_eig_solve(hipStream_t st, GroupEig& ge, const GroupDueMask& due, int max_sweeps, int ahead,
                    int* sweeps_out, int* code_out) {
  const int count = ge.count;
  const GEigDesc* tab = static_cast<const GEigDesc*>(ge.dtab);
  const int* offs = reinterpret_cast<const int*>(static_cast<const char*>(ge.dtab) + sizeof(GEigDesc) * kGroupMax);
  auto off_of = [&](int kind) { return offs + kind * (count + 1); };
  auto wgs_of = [&](int kind) { return ge.off[kind * (count + 1) + count]; };
  int* hactive = ge.dflags;            // [0]: descents still sweeping
  int* hsweeps = ge.dflags + 1;        // [1 + i]: sweeps of descent i
  ge.hflags[0] = 0;
  auto read_out = [&]() {
    for (int i = 0; i < count; ++i)
      if (due_mask_bit(due, i)) {
        sweeps_out[i] = __atomic_load_n(&ge.hflags[1 + i], __ATOMIC_ACQUIRE);
        if (code_out) code_out[i] = __atomic_load_n(&ge.hflags[1 + kGroupMax + i], __ATOMIC_ACQUIRE);
      }
  };
  // descents with N = 32 solve whole in one workgroup each, warm start
  // included, to completion
  if (ge.nsmall > 0) kg_small_solve<<<count, 256, 0, st>>>(tab, count, due, max_sweeps, hsweeps);
  if (ge.nsmall == count) {
    CMX_HIP(hipGetLastError());
    CMX_HIP(hipStreamSynchronize(st));
    read_out();
    return 0;
  }
  kg_start<<<1, 256, 0, st>>>(tab, count, due, max_sweeps, ge.dactive, hactive, hsweeps);
  kg_first<<<wgs_of(0), 256, 0, st>>>(tab, off_of(0), count);
  CMX_HIP(hipGetLastError());
  // sweeps: every batch is one sweep of the largest descent (p_max - 1
  // rounds; smaller descents complete at least one sweep in it).  `ahead`
  // batches (the longest run any descent makes before its first convergence
  // test) are queued before the host first waits; then one batch per wait
  // until no descent sweeps any more.  Rounds of descents that have stopped
  // return at once.
  // With short sweeps (small n) several are queued per wait, about kWaitRounds
  // rounds, since a round of stopped descents costs little and a wait much.
  constexpr int kWaitRounds = 8;
  const int rounds = ge.pmax - 1;
  const int per_wait = std::max(1, kWaitRounds / rounds);
  int rg = 0;
  auto queue_rounds = [&](int nr) -> int {
    for (int r = 0; r < nr; ++r, ++rg)
      kg_round<<<wgs_of(1), 256, 0, st>>>(tab, off_of(0), off_of(1), count, ge.uq, ge.ur, rg, max_sweeps,
                                          ge.dactive, hactive, hsweeps);
    CMX_HIP(hipGetLastError());
    return 0;
  };
  auto queue_batch = [&]() -> int { return queue_rounds(rounds); };
  // The first batch ends one round into the next sweep: a sweep is decided
  // at the start of the round after it, so every wait then follows the
  // decision on the last sweep queued before it.
  int queued = 0;
  for (; queued < std::min(std::max(ahead, per_wait), max_sweeps); ++queued)
    if (int rc = queue_batch()) return rc;
  if (int rc = queue_rounds(1)) return rc;
  for (;;) {
    CMX_HIP(hipStreamSynchronize(st));
    if (__atomic_load_n(&ge.hflags[0], __ATOMIC_ACQUIRE) <= 0) break;
    if (queued >= max_sweeps + per_wait)
      return fail(-3, "grouped eigensolve: descents still sweeping past the sweep limit");
    for (int b = 0; b < per_wait; ++b, ++queued)
      if (int rc = queue_batch()) return rc;
  }
  kg_rank<<<wgs_of(2), 256, 0, st>>>(tab, off_of(2), count);
  kg_colsign<<<wgs_of(3), 256, 0, st>>>(tab, off_of(3), count);
  kg_permute<<<wgs_of(4), 256, 0, st>>>(tab, off_of(4), count);
  CMX_HIP(hipGetLastError());
  read_out();
  return 0;
}

}  // namespace cmx
