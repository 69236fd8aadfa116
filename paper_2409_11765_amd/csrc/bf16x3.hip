// Sampling product y = (B D) z (eq. (1); Sec. 3.1 rewrites the sampling of
// all lambda points as one matrix product) as three bfloat16 products with
// float32 accumulation, for large n.
//
// Every operand value x is split once per generation into a bfloat16 pair
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi), both rounded to nearest
// even), which keeps about 16 significant bits.  The product keeps the three
// significant terms hi*hi + hi*lo + lo*hi (the dropped lo*lo term is below
// 2^-16 of the product) on v_mfma_f32_32x32x16_bf16.
//
// Two launches:
//  * k_split: B D (float32, column-major, m contiguous) and Z (float32,
//    column-major, k contiguous) into bf16 hi / lo arrays in a slab-major
//    layout, so that the product's k-slabs are contiguous runs of memory;
//  * k_bf16x3: 256 x 128 output tiles, 4 waves of 128 x 64, k-slabs of 32
//    double-buffered in LDS (one barrier per slab), global loads two slabs
//    ahead, LDS operand reads one k-step ahead of the MFMAs that use them.
//
// Split layout: an operand with R rows (output rows m of B D, or columns j of
// Z) and K reduction indices is held as two arrays (hi, lo) of shape
// [Kp / 32][Rp][32] with Kp = K rounded up to 64 and Rp = R rounded up to the
// tile: element (r, k) sits at ((k / 32) * Rp + r) * 32 + k % 32.  Padding
// rows and padding k are zero, so the product has no edge cases inside its
// k-loop and rows past the edge only feed outputs that are not stored.
#include <algorithm>

#include "internal.h"

namespace cmx {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kSlab = 32;             // k values per slab
constexpr int kTM = 256, kTN = 128;   // output tile (rows of B D, columns of Z)
constexpr int kPitch = kSlab + 8;     // LDS row pitch in bf16 (80 bytes: 16 rows hit 16 distinct bank groups)

// float32 -> bfloat16, round to nearest even; inf and nan keep their upper half
__device__ __forceinline__ unsigned short f2bf(float x) {
  const unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<unsigned short>(u >> 16);
  return static_cast<unsigned short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(static_cast<unsigned>(h) << 16); }

// eight float32 values -> eight (hi, lo) pairs, stored as two 16-byte runs
__device__ __forceinline__ void split8(const float (&v)[8], unsigned short* __restrict__ hi,
                                       unsigned short* __restrict__ lo) {
  unsigned short h[8], l[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    h[c] = f2bf(v[c]);
    l[c] = f2bf(v[c] - bf2f(h[c]));
  }
  uint4 ph, pl;
  ph.x = h[0] | (static_cast<unsigned>(h[1]) << 16);
  ph.y = h[2] | (static_cast<unsigned>(h[3]) << 16);
  ph.z = h[4] | (static_cast<unsigned>(h[5]) << 16);
  ph.w = h[6] | (static_cast<unsigned>(h[7]) << 16);
  pl.x = l[0] | (static_cast<unsigned>(l[1]) << 16);
  pl.y = l[2] | (static_cast<unsigned>(l[3]) << 16);
  pl.z = l[4] | (static_cast<unsigned>(l[5]) << 16);
  pl.w = l[6] | (static_cast<unsigned>(l[7]) << 16);
  *reinterpret_cast<uint4*>(hi) = ph;
  *reinterpret_cast<uint4*>(lo) = pl;
}

struct SplitArgs {
  int M, N, K, Mp, Np, nslab;
  const float* BD;
  int ldbd;
  const float* Z;
  int ldz;
  unsigned short *Ah, *Al, *Bh, *Bl;
  int blocks_a;  // workgroups [0, blocks_a) split B D, the rest split Z
};

// Workgroups [0, blocks_a): one 64 (m) x 32 (k) block of B D each, transposed
// through LDS (reads of 64 consecutive m per wave, writes of 8 consecutive k
// per thread).  The rest: 64 columns of one k-slab of Z each (8 consecutive k
// per thread, already contiguous in Z).
__global__ void __launch_bounds__(256) k_split(SplitArgs a) {
  const int t = threadIdx.x;
  if (static_cast<int>(blockIdx.x) < a.blocks_a) {
    __shared__ float T[kSlab][64 + 1];
    const int mblocks = a.Mp / 64;
    const int mb = blockIdx.x % mblocks, kt = blockIdx.x / mblocks;
    const int m0 = mb * 64, k0 = kt * kSlab;
    {
      const int m = m0 + (t & 63);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int kk = (t >> 6) + 4 * i, k = k0 + kk;
        T[kk][t & 63] = (m < a.M && k < a.K) ? a.BD[static_cast<int64_t>(k) * a.ldbd + m] : 0.0f;
      }
    }
    __syncthreads();
    const int r = t >> 2, kc = (t & 3) * 8;
    float v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = T[kc + c][r];
    const int64_t o = (static_cast<int64_t>(kt) * a.Mp + m0 + r) * kSlab + kc;
    split8(v, a.Ah + o, a.Al + o);
  } else {
    const int64_t c = static_cast<int64_t>(blockIdx.x - a.blocks_a) * 256 + t;
    if (c >= static_cast<int64_t>(a.nslab) * a.Np * 4) return;
    const int kc = static_cast<int>(c & 3) * 8;
    const int j = static_cast<int>((c >> 2) % a.Np);
    const int kt = static_cast<int>((c >> 2) / a.Np);
    const int k = kt * kSlab + kc;
    float v[8];
    const float* src = a.Z + static_cast<int64_t>(j) * a.ldz + k;
    if (j < a.N && k + 8 <= a.K) {
      const float4 x0 = *reinterpret_cast<const float4*>(src);
      const float4 x1 = *reinterpret_cast<const float4*>(src + 4);
      v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
      v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (j < a.N && k + e < a.K) ? src[e] : 0.0f;
    }
    const int64_t o = (static_cast<int64_t>(kt) * a.Np + j) * kSlab + kc;
    split8(v, a.Bh + o, a.Bl + o);
  }
}

struct ProdArgs {
  int M, N, Mp, Np, nk, tiles_m;
  const unsigned short *Ah, *Al, *Bh, *Bl;
  float* Y;
  int ldy;
};

// One stage of LDS: hi and lo slabs of A (256 rows) and B (128 rows).
struct Stage {
  unsigned short ah[kTM * kPitch], al[kTM * kPitch], bh[kTN * kPitch], bl[kTN * kPitch];
};

// The slab's 16-byte pieces of this thread: A hi and lo rows (4 each), then
// B hi and lo rows (2 each).  Piece p of a 16-byte-per-piece run covers row
// p / 4, k 8 (p % 4) .. 8 (p % 4) + 7.
struct Pieces {
  u32x4 v[12];
};

__device__ __forceinline__ void load_slab(const ProdArgs& a, int kt, int m0, int n0, Pieces& P) {
  const int t = threadIdx.x;
  const int64_t abase = (static_cast<int64_t>(kt) * a.Mp + m0) * kSlab;
  const int64_t bbase = (static_cast<int64_t>(kt) * a.Np + n0) * kSlab;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t o = abase + (t + 256 * i) * 8;
    P.v[i] = *reinterpret_cast<const u32x4*>(a.Ah + o);
    P.v[4 + i] = *reinterpret_cast<const u32x4*>(a.Al + o);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int64_t o = bbase + (t + 256 * i) * 8;
    P.v[8 + i] = *reinterpret_cast<const u32x4*>(a.Bh + o);
    P.v[10 + i] = *reinterpret_cast<const u32x4*>(a.Bl + o);
  }
}

__device__ __forceinline__ void store_slab(Stage& S, const Pieces& P) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = t + 256 * i, o = (p >> 2) * kPitch + (p & 3) * 8;
    *reinterpret_cast<u32x4*>(&S.ah[o]) = P.v[i];
    *reinterpret_cast<u32x4*>(&S.al[o]) = P.v[4 + i];
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int p = t + 256 * i, o = (p >> 2) * kPitch + (p & 3) * 8;
    *reinterpret_cast<u32x4*>(&S.bh[o]) = P.v[8 + i];
    *reinterpret_cast<u32x4*>(&S.bl[o]) = P.v[10 + i];
  }
}

// Operands of one 16-wide k-step of this wave's 128 x 64 block.
struct Frags {
  bf16x8 ah[4], al[4], bh[2], bl[2];
};

__device__ __forceinline__ void read_frags(const Stage& S, int step, int wm, int wn, int row, int kh, Frags& F) {
  const int ko = step * 16 + kh;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = (wm * 128 + i * 32 + row) * kPitch + ko;
    F.ah[i] = *reinterpret_cast<const bf16x8*>(&S.ah[o]);
    F.al[i] = *reinterpret_cast<const bf16x8*>(&S.al[o]);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int o = (wn * 64 + j * 32 + row) * kPitch + ko;
    F.bh[j] = *reinterpret_cast<const bf16x8*>(&S.bh[o]);
    F.bl[j] = *reinterpret_cast<const bf16x8*>(&S.bl[o]);
  }
}

// The 24 MFMAs of one k-step: per output block lo*hi, then hi*lo, then hi*hi
// (small terms first); the blocks interleave so that no MFMA waits on the one
// before it.
__device__ __forceinline__ void mma_step(const Frags& F, floatx16 (&acc)[4][2]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.al[i], F.bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.ah[i], F.bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.ah[i], F.bh[j], acc[i][j], 0, 0, 0);
}

__global__ void __launch_bounds__(256) k_bf16x3(ProdArgs a) {
  __shared__ Stage st[2];
  // a launch with a multiple of 8 workgroups gives each XCD (blockIdx % 8) a
  // contiguous run of tiles, m fastest: its workgroups then share B D slabs
  // and pairs of Z slabs in that XCD's L2
  int tile = blockIdx.x;
  if ((gridDim.x & 7) == 0) tile = (tile & 7) * (gridDim.x >> 3) + (tile >> 3);
  const int m0 = (tile % a.tiles_m) * kTM, n0 = (tile / a.tiles_m) * kTN;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  const int row = lane & 31, kh = (lane >> 5) * 8;
  // Software pipeline over slabs (LDS buffer kt % 2 holds slab kt):
  //  * global: a pass loads slab kt + 2 into one register set while the other
  //    holds slab kt + 1, which the pass stores into the idle LDS buffer (past
  //    the end the last slab is loaded again, so every load is unconditional
  //    and in bounds);
  //  * LDS: the operands of a slab's second k-step are read under the MFMAs
  //    of its first, and those of the next slab's first k-step, right after
  //    the barrier, under the MFMAs of its second.
  // The scheduling barriers keep each group of reads ahead of the MFMAs that
  // hide it.
  Pieces P0, P1;
  Frags F0, F1;
  load_slab(a, 0, m0, n0, P0);
  load_slab(a, min(1, a.nk - 1), m0, n0, P1);
  store_slab(st[0], P0);
  __syncthreads();
  read_frags(st[0], 0, wm, wn, row, kh, F0);
  for (int kt = 0; kt < a.nk; kt += 2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // pass kt + h: slab kt + h in st[h]
      load_slab(a, min(kt + h + 2, a.nk - 1), m0, n0, h == 0 ? P0 : P1);
      read_frags(st[h], 1, wm, wn, row, kh, F1);
      __builtin_amdgcn_sched_barrier(0);
      mma_step(F0, acc);
      store_slab(st[h ^ 1], h == 0 ? P1 : P0);
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
      read_frags(st[h ^ 1], 0, wm, wn, row, kh, F0);
      __builtin_amdgcn_sched_barrier(0);
      mma_step(F1, acc);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // acc[i][j][r] holds row (r / 4) * 8 + (lane / 32) * 4 + r % 4 of the
  // 32 x 32 block, column lane % 32: four consecutive rows per 16-byte store
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 64 + j * 32 + row;
      if (col >= a.N) continue;
      float* yc = a.Y + static_cast<int64_t>(col) * a.ldy;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r0 = m0 + wm * 128 + i * 32 + q * 8 + (lane >> 5) * 4;
        if (r0 + 4 <= a.M) {
          *reinterpret_cast<float4*>(yc + r0) =
              make_float4(acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (r0 + e < a.M) yc[r0 + e] = acc[i][j][4 * q + e];
        }
      }
    }
}

void split_dims(int n, int lam, int* Mp, int* Np, int* Kp) {
  *Mp = round_up(std::max(n, 1), kTM);
  *Np = round_up(std::max(lam, 1), kTN);
  *Kp = round_up(std::max(n, 1), 2 * kSlab);  // an even number of slabs: the k-loop takes them in pairs
}

}  // namespace

size_t bf16x3_work_bytes(int n, int lam) {
  int Mp, Np, Kp;
  split_dims(n, lam, &Mp, &Np, &Kp);
  return 2ull * 2ull * static_cast<size_t>(Kp) * (static_cast<size_t>(Mp) + Np);
}

hipError_t launch_sample_gemm_bf16x3(hipStream_t st, int n, int lam, const float* BD, int ldbd, const float* Z,
                                     int ldz, float* Y, int ldy, void* work, KTimer* kt, int kid) {
  if ((ldbd & 3) || (ldz & 3) || (ldy & 3) || ldbd < n || ldz < n || ldy < n || !work) return hipErrorInvalidValue;
  if (n <= 0 || lam <= 0) return hipSuccess;
  int Mp, Np, Kp;
  split_dims(n, lam, &Mp, &Np, &Kp);
  const size_t slab_a = static_cast<size_t>(Kp) * Mp, slab_b = static_cast<size_t>(Kp) * Np;
  unsigned short* w = static_cast<unsigned short*>(work);
  SplitArgs s{n, lam, n, Mp, Np, Kp / kSlab, BD, ldbd, Z, ldz, w, w + slab_a, w + 2 * slab_a, w + 2 * slab_a + slab_b, 0};
  s.blocks_a = (Mp / 64) * (Kp / kSlab);
  const int64_t chunks_b = static_cast<int64_t>(Kp / kSlab) * Np * 4;  // 8 k values each
  const int blocks_b = static_cast<int>((chunks_b + 255) / 256);
  k_split<<<s.blocks_a + blocks_b, 256, 0, st>>>(s);
  ProdArgs p{n, lam, Mp, Np, Kp / kSlab, Mp / kTM, s.Ah, s.Al, s.Bh, s.Bl, Y, ldy};
  timed_launch(kt, kid, k_bf16x3, (Mp / kTM) * (Np / kTN), 256, st, p);
  return hipGetLastError();
}

}  // namespace cmx
