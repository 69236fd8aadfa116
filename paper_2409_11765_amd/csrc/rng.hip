// Counter-based normal sampler: Philox4x32-10 (Salmon et al., SC'11) and the
// Box-Muller transform give the z_k ~ N(0, I) of eq. (1) (Sec. 2.1).
//
// Element (i, k) of the n x lambda matrix Z comes from the Philox block with
// counter (i / 4, k, generation, restart) and key = 64-bit seed: words
// (r0, r1) give rows 4j, 4j+1 and words (r2, r3) rows 4j+2, 4j+3.  Because
// the stream is a pure function of (seed, restart, generation, k, i), a
// generation can be replayed, resumed or split over devices without state.
// One thread produces one 4-row block and writes it with a single vector
// store, so consecutive threads write consecutive 16/32-byte segments.
#include "internal.h"

namespace cmx {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(kPhiloxM0, c.x), lo0 = kPhiloxM0 * c.x;
    const uint32_t hi1 = __umulhi(kPhiloxM1, c.z), lo1 = kPhiloxM1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return c;
}

// (u + 1/2) / 2^32, strictly inside (0, 1)
__device__ __forceinline__ double unit_open(uint32_t u) {
  return (static_cast<double>(u) + 0.5) * 2.3283064365386962890625e-10;
}

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double rho = sqrt(-2.0 * log(unit_open(a)));
  double s, c;
  sincospi(2.0 * unit_open(b), &s, &c);
  z0 = rho * c;
  z1 = rho * s;
}

template <typename T>
__device__ __forceinline__ void normals_body(int bx, T* __restrict__ Z, int ldz, int n, int lam, uint32_t k0,
                                             uint32_t k1, uint32_t restart, const DevScalars* __restrict__ sc) {
  const int nb = (n + 3) >> 2;
  const int64_t idx = static_cast<int64_t>(bx) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nb) * lam) return;
  const int k = static_cast<int>(idx / nb);
  const int j = static_cast<int>(idx - static_cast<int64_t>(k) * nb);
  const uint32_t gen = static_cast<uint32_t>(sc->gen);
  const uint4 r = philox4x32_10(make_uint4(static_cast<uint32_t>(j), static_cast<uint32_t>(k), gen,
                                           restart),
                                k0, k1);
  double z[4];
  box_muller(r.x, r.y, z[0], z[1]);
  box_muller(r.z, r.w, z[2], z[3]);
  T* dst = Z + static_cast<int64_t>(k) * ldz + 4 * j;
  if (4 * j + 3 < n) {
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float4*>(dst) = make_float4(static_cast<float>(z[0]), static_cast<float>(z[1]),
                                                    static_cast<float>(z[2]), static_cast<float>(z[3]));
    } else {
      reinterpret_cast<double2*>(dst)[0] = make_double2(z[0], z[1]);
      reinterpret_cast<double2*>(dst)[1] = make_double2(z[2], z[3]);
    }
  } else {
    for (int q = 0; q < 4 && 4 * j + q < n; ++q) dst[q] = static_cast<T>(z[q]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_normals(T* __restrict__ Z, int ldz, int n, int lam,
                                                 uint32_t k0, uint32_t k1, uint32_t restart,
                                                 const DevScalars* __restrict__ sc) {
  normals_body<T>(blockIdx.x, Z, ldz, n, lam, k0, k1, restart, sc);
}

// the normals of every descent of a group (float32)
__global__ void __launch_bounds__(256) kg_normals(const GFront* __restrict__ g, const int* __restrict__ off,
                                                  int count) {
  const int i = group_find(off, count, blockIdx.x);
  const GFront& e = g[i];
  normals_body<float>(blockIdx.x - off[i], e.Z, e.ldn, e.n, e.lam, e.k0, e.k1, e.restart, e.sc);
}

// Initial mean of a descent: uniform in [lo, hi]^n (Sec. 4.1); coordinate i
// uses word i % 4 of the Philox block (i / 4, 0, 0xFFFFFFFF, restart).
__global__ void k_init_mean(double* __restrict__ m, int n, double lo, double hi, uint32_t k0,
                            uint32_t k1, uint32_t restart) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * j >= n) return;
  const uint4 r = philox4x32_10(make_uint4(static_cast<uint32_t>(j), 0u, 0xFFFFFFFFu, restart), k0, k1);
  const uint32_t w[4] = {r.x, r.y, r.z, r.w};
  for (int q = 0; q < 4 && 4 * j + q < n; ++q) m[4 * j + q] = lo + (hi - lo) * unit_open(w[q]);
}

}  // namespace

hipError_t launch_normals(hipStream_t st, void* Z, bool fp64, int ldz, int n, int lam,
                          uint64_t seed, uint32_t restart, const DevScalars* sc) {
  if ((ldz & 3) != 0) return hipErrorInvalidValue;  // vector stores need 4-aligned columns
  const int nb = (n + 3) / 4;
  const int64_t total = static_cast<int64_t>(nb) * lam;
  const int blocks = static_cast<int>((total + 255) / 256);
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  if (fp64)
    k_normals<double><<<blocks, 256, 0, st>>>(static_cast<double*>(Z), ldz, n, lam, k0, k1, restart, sc);
  else
    k_normals<float><<<blocks, 256, 0, st>>>(static_cast<float*>(Z), ldz, n, lam, k0, k1, restart, sc);
  return hipGetLastError();
}

hipError_t launch_group_normals(hipStream_t st, const GFront* g, const int* off, int count, int wgs) {
  if (wgs > 0) kg_normals<<<wgs, 256, 0, st>>>(g, off, count);
  return hipGetLastError();
}

hipError_t launch_init_mean(hipStream_t st, double* m, int n, double lo, double hi, uint64_t seed,
                            uint32_t restart) {
  const int nb = (n + 3) / 4;
  k_init_mean<<<ceil_div(nb, 256), 256, 0, st>>>(m, n, lo, hi, static_cast<uint32_t>(seed),
                                                 static_cast<uint32_t>(seed >> 32), restart);
  return hipGetLastError();
}

}  // namespace cmx
