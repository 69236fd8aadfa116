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
//     round-r tiles its next pair needs instead of waiting for them.
//     Sweeps stop when the off-diagonal Frobenius norm of A falls below
//     1e-13 of its total norm (summed per tile by the last round).
//  3. B = B_old V, D = sqrt(diag A), then the pairs are canonicalised like the
//     oracle: ascending eigenvalues, each column's largest-magnitude entry
//     positive.  B D is also written in the sampling precision.
#include <algorithm>
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
// refined by Newton steps: one step gives about 1e-14, two give full double
// precision.
__device__ __forceinline__ double rcp_nr1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return y * fma(-x, y, 2.0);
}
__device__ __forceinline__ double rsq_nr1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ double rsq_nr2(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y * fma(-0.5 * x * y, y, 1.5);
}

// Jacobi rotation J = [[c, s], [-s, c]] on (a, b) with (J^T S J)_ab = 0
// (Golub & Van Loan, sym.schur2): t = sign(delta) 2 d / (|delta| + sqrt(delta^2 + 4 d^2))
// with delta = S_bb - S_aa, d = S_ab; c = 1/sqrt(1 + t^2), s = t c; the
// identity when |d| <= thr.  Branch free, so the callers' loads issue up front
// and two rotations interleave.  t is accurate to about 1e-14 relative (it
// only decides how well the entry is annihilated); c is refined to full
// precision because c^2 (1 + t^2) = 1 is what keeps Q orthogonal.
__device__ __forceinline__ void jacobi_rotation(double saa, double sbb, double d, double thr, double& c,
                                                double& s) {
  // |d| <= thr gives d' = 0 and hence t = 0; the floor on h2 keeps every
  // intermediate finite, so no branch is needed
  const double dd = fabs(d) > thr ? d : 0.0;
  const double delta = sbb - saa;
  const double h2 = fmax(fma(delta, delta, 4.0 * dd * dd), 1e-280);
  const double h = h2 * rsq_nr1(h2);
  const double t = (delta >= 0.0 ? 2.0 : -2.0) * dd * rcp_nr1(fabs(delta) + h);
  c = rsq_nr2(fma(t, t, 1.0));
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

// load a column-major 32x32 Q (global) into LDS rows
__device__ __forceinline__ void load_q(const double* __restrict__ q, double* Q) {
  for (int idx = threadIdx.x; idx < kS * kS; idx += 256) Q[(idx % kS) * kLD + idx / kS] = q[idx];
}

// X <- Q1^T A[{P1 blocks}, {P2 blocks}] Q2 for round r (W is scratch); all in LDS
__device__ void tile_transform(const double* __restrict__ A, int N, int p, int r, int P1, int P2,
                               const double* Q1, const double* Q2, double* X, double* W) {
  int I1, J1, I2, J2;
  block_pair(p, r, P1, I1, J1);
  block_pair(p, r, P2, I2, J2);
  for (int idx = threadIdx.x; idx < kS * kS; idx += 256) {
    const int rr = idx % kS, c = idx / kS;
    X[rr * kLD + c] = A[static_cast<int64_t>(gidx(I2, J2, c)) * N + gidx(I1, J1, rr)];
  }
  __syncthreads();
  mm32<false>(X, Q2, W);  // W = X Q2
  __syncthreads();
  mm32<true>(Q1, W, X);   // X = Q1^T W
  __syncthreads();
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

// One inner round: every thread owns one 2x2 block (rotation x, rotation y),
// recomputes the two rotations it needs, updates its block of S into the
// other buffer and rows r0, r1 of Q for rotation x.
template <bool INTRA>
__device__ __forceinline__ void inner_round(const double* S, double* Sn, double* Q, double thr, int rr, int x,
                                            int y) {
  int ax, bx, ay, by;
  pair_idx<INTRA>(rr, x, ax, bx);
  pair_idx<INTRA>(rr, y, ay, by);
  const int r0 = 2 * y, r1 = 2 * y + 1;
  const double xaa = S[ax * kLD + ax], xbb = S[bx * kLD + bx], xab = S[ax * kLD + bx];
  const double yaa = S[ay * kLD + ay], ybb = S[by * kLD + by], yab = S[ay * kLD + by];
  const double m00 = S[ax * kLD + ay], m01 = S[ax * kLD + by];
  const double m10 = S[bx * kLD + ay], m11 = S[bx * kLD + by];
  const double q0a = Q[r0 * kLD + ax], q0b = Q[r0 * kLD + bx];
  const double q1a = Q[r1 * kLD + ax], q1b = Q[r1 * kLD + bx];
  double cx, sx, cy, sy;
  jacobi_rotation(xaa, xbb, xab, thr, cx, sx);
  jacobi_rotation(yaa, ybb, yab, thr, cy, sy);
  // S_xy <- J_x^T S_xy J_y,  J = [[c, s], [-s, c]] on (a, b)
  const double p00 = m00 * cy - m01 * sy, p01 = m00 * sy + m01 * cy;
  const double p10 = m10 * cy - m11 * sy, p11 = m10 * sy + m11 * cy;
  const double n00 = cx * p00 - sx * p10, n11 = sx * p01 + cx * p11;
  double n01 = cx * p01 - sx * p11, n10 = sx * p00 + cx * p10;
  if (x == y) {  // the annihilated entry is exactly zero
    n01 = 0.0;
    n10 = 0.0;
  }
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
// barrier per inner round.
__device__ void rotate_pair(double* S0, double* S1, double* Q, double thr, bool with_intra,
                            double* __restrict__ qout) {
  const int t = threadIdx.x;
  for (int idx = t; idx < kS * kS; idx += 256) Q[(idx % kS) * kLD + idx / kS] = (idx % kS == idx / kS) ? 1.0 : 0.0;
  const int x = t % (kS / 2), y = t / (kS / 2);
  double* Sa = S0;
  double* Sb = S1;
  __syncthreads();
  if (with_intra) {
    for (int rr = 0; rr < kNB - 1; ++rr) {
      inner_round<true>(Sa, Sb, Q, thr, rr, x, y);
      double* tmp = Sa;
      Sa = Sb;
      Sb = tmp;
      __syncthreads();
    }
  }
  for (int rr = 0; rr < kNB; ++rr) {
    inner_round<false>(Sa, Sb, Q, thr, rr, x, y);
    double* tmp = Sa;
    Sa = Sb;
    Sb = tmp;
    __syncthreads();
  }
  for (int idx = t; idx < kS * kS; idx += 256) qout[idx] = Q[(idx % kS) * kLD + idx / kS];
  __syncthreads();
}

// First pair solves of a descent's eigensolve: round 0 (with the intra-block
// rotations) straight from A.
__global__ void __launch_bounds__(256) k_jac_first(const double* __restrict__ A, int N, int p,
                                                   const double* __restrict__ scale, double* __restrict__ Qg) {
  __shared__ double lds[3 * kS * kLD];
  double* S0 = lds;
  double* S1 = lds + kS * kLD;
  double* Q = lds + 2 * kS * kLD;
  const int P = blockIdx.x;
  int I, J;
  block_pair(p, 0, P, I, J);
  for (int idx = threadIdx.x; idx < kS * kS; idx += 256) {
    const int r = idx % kS, c = idx / kS;
    S0[r * kLD + c] = A[static_cast<int64_t>(gidx(I, J, c)) * N + gidx(I, J, r)];
  }
  __syncthreads();
  rotate_pair(S0, S1, Q, 2.2e-16 * (*scale), true, Qg + static_cast<int64_t>(P) * kS * kS);
}

// One outer round r: workgroups [0, q) run the pair solves of the next round
// (r + 1, or round 0 of the next sweep after the last round); workgroups
// [q, q + q(q+1)/2) write the round-r lower tiles Q_P1^T A_cur Q_P2 of A into
// A_next (mirrored) and their off-diagonal / total squared norms into
// tilepart; the rest update 32-row pieces of V with V Q_P.
__global__ void __launch_bounds__(256) k_jac_round(const double* __restrict__ Acur, double* __restrict__ Anext,
                                                   double* __restrict__ V, const double* __restrict__ Qcur,
                                                   double* __restrict__ Qnext, int N, int r,
                                                   const double* __restrict__ scale, double* __restrict__ tilepart) {
  __shared__ double lds[5 * kS * kLD];
  double* QA = lds;
  double* QB = lds + kS * kLD;
  double* X = lds + 2 * kS * kLD;
  double* W = lds + 3 * kS * kLD;
  double* S = lds + 4 * kS * kLD;
  const int p = N / kNB, q = p / 2;
  const int ntiles = q * (q + 1) / 2;
  const int t = threadIdx.x;
  int b = blockIdx.x;
  if (b < q) {
    // ---- pair solve of the next round, from recomputed round-r tiles:
    // the tiles (Pa,Pa), (Pb,Pb), (Pa,Pb) and both Q's are fetched at once
    // (the last two tiles wait in registers), transformed one after the
    // other, and the next pair's S assembled from them.
    const bool wrap = (r + 1 == p - 1);
    const int rn = wrap ? 0 : r + 1;
    int In, Jn;
    block_pair(p, rn, b, In, Jn);
    const int Pa = pair_of(p, r, In), Pb = pair_of(p, r, Jn);
    int Ia, Ja, Ib, Jb;
    block_pair(p, r, Pa, Ia, Ja);
    block_pair(p, r, Pb, Ib, Jb);
    const int pi = (In == Ia) ? 0 : kNB, pj = (Jn == Ib) ? 0 : kNB;
    const double* qa = Qcur + static_cast<int64_t>(Pa) * kS * kS;
    const double* qb = Qcur + static_cast<int64_t>(Pb) * kS * kS;
    constexpr int PER = kS * kS / 256;
    double t2[PER], t3[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = t + 256 * k, rr = idx % kS, c = idx / kS;
      QA[rr * kLD + c] = qa[idx];
      QB[rr * kLD + c] = qb[idx];
      X[rr * kLD + c] = Acur[static_cast<int64_t>(gidx(Ia, Ja, c)) * N + gidx(Ia, Ja, rr)];
      t2[k] = Acur[static_cast<int64_t>(gidx(Ib, Jb, c)) * N + gidx(Ib, Jb, rr)];
      t3[k] = Acur[static_cast<int64_t>(gidx(Ib, Jb, c)) * N + gidx(Ia, Ja, rr)];
    }
    __syncthreads();
    mm32<false>(X, QA, W);
    __syncthreads();
    mm32<true>(QA, W, X);  // X = Qa^T A[Pa,Pa] Qa
    __syncthreads();
    if (Pa == Pb) {
      // both blocks of the next pair come from one round-r pair (p = 2)
      const int pjj = (Jn == Ia) ? 0 : kNB;
      for (int idx = t; idx < kS * kS; idx += 256) {
        const int rr = idx % kS, c = idx / kS;
        const int sr = rr < kNB ? pi + rr : pjj + rr - kNB;
        const int sc = c < kNB ? pi + c : pjj + c - kNB;
        S[rr * kLD + c] = X[sr * kLD + sc];
      }
    } else {
      for (int idx = t; idx < kNB * kNB; idx += 256) {
        const int rr = idx % kNB, c = idx / kNB;
        S[rr * kLD + c] = X[(pi + rr) * kLD + pi + c];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = t + 256 * k;
        X[(idx % kS) * kLD + idx / kS] = t2[k];
      }
      __syncthreads();
      mm32<false>(X, QB, W);
      __syncthreads();
      mm32<true>(QB, W, X);  // X = Qb^T A[Pb,Pb] Qb
      __syncthreads();
      for (int idx = t; idx < kNB * kNB; idx += 256) {
        const int rr = idx % kNB, c = idx / kNB;
        S[(kNB + rr) * kLD + kNB + c] = X[(pj + rr) * kLD + pj + c];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = t + 256 * k;
        X[(idx % kS) * kLD + idx / kS] = t3[k];
      }
      __syncthreads();
      mm32<false>(X, QB, W);
      __syncthreads();
      mm32<true>(QA, W, X);  // X = Qa^T A[Pa,Pb] Qb
      __syncthreads();
      for (int idx = t; idx < kNB * kNB; idx += 256) {
        const int rr = idx % kNB, c = idx / kNB;
        const double v = X[(pi + rr) * kLD + pj + c];
        S[rr * kLD + kNB + c] = v;
        S[(kNB + c) * kLD + rr] = v;
      }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(2);  // the pair solves are the round's critical path
    rotate_pair(S, X, W, 2.2e-16 * (*scale), wrap, Qnext + static_cast<int64_t>(b) * kS * kS);
    return;
  }
  b -= q;
  if (b < ntiles) {
    // ---- round-r tile of A into A_next
    int P1 = static_cast<int>((sqrtf(8.0f * b + 1.0f) - 1.0f) * 0.5f);
    while ((P1 + 1) * (P1 + 2) / 2 <= b) ++P1;
    while (P1 * (P1 + 1) / 2 > b) --P1;
    const int P2 = b - P1 * (P1 + 1) / 2;
    load_q(Qcur + static_cast<int64_t>(P1) * kS * kS, QA);
    load_q(Qcur + static_cast<int64_t>(P2) * kS * kS, QB);
    __syncthreads();
    tile_transform(Acur, N, p, r, P1, P2, QA, QB, X, W);
    int I1, J1, I2, J2;
    block_pair(p, r, P1, I1, J1);
    block_pair(p, r, P2, I2, J2);
    double off = 0.0, tot = 0.0, dmax = 0.0;
    for (int idx = t; idx < kS * kS; idx += 256) {
      const int rr = idx % kS, c = idx / kS;
      const int gr = gidx(I1, J1, rr), gc = gidx(I2, J2, c);
      const double v = X[rr * kLD + c];
      Anext[static_cast<int64_t>(gc) * N + gr] = v;
      tot += v * v;
      if (gr != gc) off += v * v;
      else dmax = fmax(dmax, fabs(v));
    }
    if (P1 != P2) {
      for (int idx = t; idx < kS * kS; idx += 256) {
        const int c = idx % kS, rr = idx / kS;  // consecutive threads -> consecutive rows of the mirror
        Anext[static_cast<int64_t>(gidx(I1, J1, rr)) * N + gidx(I2, J2, c)] = X[rr * kLD + c];
      }
      off *= 2.0;
      tot *= 2.0;
    }
    double* red = W;  // W is free after the transform: 3 x 256 partial sums
    red[t] = off;
    red[256 + t] = tot;
    red[512 + t] = dmax;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
      if (t < s2) {
        red[t] += red[t + s2];
        red[256 + t] += red[256 + t + s2];
        red[512 + t] = fmax(red[512 + t], red[512 + t + s2]);
      }
      __syncthreads();
    }
    if (t == 0) {
      tilepart[3 * b + 0] = red[0];
      tilepart[3 * b + 1] = red[256];
      tilepart[3 * b + 2] = red[512];
    }
    return;
  }
  b -= ntiles;
  // ---- V piece: rows [32 rc, 32 rc + 32) of the columns of pair P
  const int P = b % q, rc = b / q;
  int I, J;
  block_pair(p, r, P, I, J);
  load_q(Qcur + static_cast<int64_t>(P) * kS * kS, QA);
  for (int idx = t; idx < kS * kS; idx += 256) {
    const int rr = idx % kS, c = idx / kS;
    X[rr * kLD + c] = V[static_cast<int64_t>(gidx(I, J, c)) * N + rc * kS + rr];
  }
  __syncthreads();
  mm32<false>(X, QA, W);
  __syncthreads();
  for (int idx = t; idx < kS * kS; idx += 256) {
    const int rr = idx % kS, c = idx / kS;
    V[static_cast<int64_t>(gidx(I, J, c)) * N + rc * kS + rr] = W[rr * kLD + c];
  }
}

// off-diagonal / total squared norms and max |diagonal| of A, per column
__global__ void __launch_bounds__(256) k_offnorm_cols(const double* __restrict__ A, int N, int n,
                                                      double* __restrict__ part) {
  __shared__ double red[3][256];
  const int c = blockIdx.x, t = threadIdx.x;
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

// reduce count (off, tot, dmax) triples in a fixed order: flags[0] = 1 if more
// sweeps are needed, flags[1] = 1 if non-finite; scale[0] = max |a_ii|
__global__ void __launch_bounds__(256) k_offnorm_final(const double* __restrict__ part, int count,
                                                       int* __restrict__ flags, double* __restrict__ scale) {
  __shared__ double red[3][256];
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
  if (t == 0) {
    const bool finite = isfinite(red[1][0]);
    flags[0] = (finite && red[0][0] > kOffTol * kOffTol * red[1][0]) ? 1 : 0;
    flags[1] = finite ? 0 : 1;
    scale[0] = red[2][0];
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
                                                  const int* __restrict__ status, DevScalars* __restrict__ sc) {
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
  if (cnt == 0) {
    sc->eig_ok = (vi > 0.0 && status[0] == 1) ? 1 : 0;
    sc->jac_sweeps = status[1];
  }
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

// ---- host side: the eigensolve as a resumable sequence, so several
// descents can advance their sweeps in lockstep with one host
// synchronisation per sweep (the convergence flag is the only value the
// host needs between sweeps; it lands in pinned host memory).

int eigen_begin(hipStream_t st, int n, const double* C, int ldc, const double* B, int ldb, EigWork& w,
                KTimer* kt) {
  const int N = w.N;
  const int64_t NN = static_cast<int64_t>(N) * N;
  w.Acur = w.A;
  w.Anext = w.A2;
  w.Qcur = w.Q;
  w.Qnext = w.Q2;
  w.sweeps = 0;
  k_fill<<<static_cast<int>((NN + 255) / 256), 256, 0, st>>>(w.Acur, NN, 0.0);
  k_fill<<<static_cast<int>((NN + 255) / 256), 256, 0, st>>>(w.Anext, NN, 0.0);
  k_identity<<<static_cast<int>((NN + 255) / 256), 256, 0, st>>>(w.V, N);
  CMX_HIP(hipGetLastError());
  kt_begin(kt, KID_EIG_GEMM);
  CMX_HIP(launch_dgemm(st, false, false, n, n, n, C, ldc, B, ldb, w.T, ldb));   // T = C B
  kt_end(kt);
  kt_begin(kt, KID_EIG_GEMM);
  CMX_HIP(launch_dgemm(st, true, false, n, n, n, B, ldb, w.T, ldb, w.Acur, N));   // A = B^T T
  kt_end(kt);
  k_offnorm_cols<<<n, 256, 0, st>>>(w.Acur, N, n, w.part);
  k_offnorm_final<<<1, 256, 0, st>>>(w.part, n, w.flags, w.scale);
  CMX_HIP(hipGetLastError());
  CMX_HIP(hipMemcpyAsync(w.hflags, w.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  w.pending = true;
  return 0;
}

__global__ void k_set_status(int* status, int code, int sweeps) {
  if (threadIdx.x == 0) {
    status[0] = code;
    status[1] = sweeps;
  }
}

int eigen_step(hipStream_t st, int n, double* B, int ldb, double* D, void* BD, bool fp64_bd, int ldbd, EigWork& w,
               DevScalars* sc, int max_sweeps, KTimer* kt, bool* done) {
  *done = false;
  const int N = w.N;
  const int p = N / kNB, q = p / 2;
  const int ntiles = q * (q + 1) / 2;
  const bool more = w.hflags[0] && !w.hflags[1];
  if (more && w.sweeps < max_sweeps) {
    if (w.sweeps == 0) {
      kt_begin(kt, KID_JACOBI);
      k_jac_first<<<q, 256, 0, st>>>(w.Acur, N, p, w.scale, w.Qcur);
      kt_end(kt);
    }
    const int round_blocks = q + ntiles + (N / kS) * q;
    for (int r = 0; r < p - 1; ++r) {
      kt_begin(kt, KID_JACOBI);
      k_jac_round<<<round_blocks, 256, 0, st>>>(w.Acur, w.Anext, w.V, w.Qcur, w.Qnext, N, r, w.scale, w.part);
      kt_end(kt);
      std::swap(w.Acur, w.Anext);
      std::swap(w.Qcur, w.Qnext);
    }
    ++w.sweeps;
    k_offnorm_final<<<1, 256, 0, st>>>(w.part, ntiles, w.flags, w.scale);
    CMX_HIP(hipGetLastError());
    CMX_HIP(hipMemcpyAsync(w.hflags, w.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    return 0;
  }
  // converged (1), sweep limit (2) or non-finite (3): finish
  k_set_status<<<1, 64, 0, st>>>(w.status, w.hflags[1] ? 3 : (w.hflags[0] ? 2 : 1), w.sweeps);
  // B_new = B V (into T), then canonical order / signs into B, D, BD
  kt_begin(kt, KID_EIG_GEMM);
  CMX_HIP(launch_dgemm(st, false, false, n, n, n, B, ldb, w.V, N, w.T, ldb));
  kt_end(kt);
  k_eig_rank<<<ceil_div(n, 256), 256, 0, st>>>(w.Acur, N, n, w.perm, w.evals, w.status, sc);
  k_colsign<<<n, 256, 0, st>>>(w.T, ldb, n, w.sign);
  dim3 grid(ceil_div(n, 256), n);
  if (fp64_bd)
    k_permute<double><<<grid, 256, 0, st>>>(w.T, ldb, n, w.perm, w.evals, w.sign, B, ldb, D,
                                            static_cast<double*>(BD), ldbd);
  else
    k_permute<float><<<grid, 256, 0, st>>>(w.T, ldb, n, w.perm, w.evals, w.sign, B, ldb, D,
                                           static_cast<float*>(BD), ldbd);
  CMX_HIP(hipGetLastError());
  w.pending = false;
  *done = true;
  return 0;
}

}  // namespace cmx
