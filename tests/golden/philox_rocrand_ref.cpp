// Known-answer generator for the oracle's Philox4x32-10: prints the raw
// output block of rocRAND's header-only philox4x32_10 engine for each
// (counter, key) read from stdin.  Used only by the CPU test suite.
//
// Input lines:  c0 c1 c2 c3 k0 k1   (decimal uint32; c1 < 2^30)
// Output lines: r0 r1 r2 r3         (decimal uint32)
//
// rocRAND's engine puts the 64-bit seed into the key, the 64-bit
// subsequence into counter words 2..3 and offset/4 into counter words 0..1.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const unsigned long long seed = (k1 << 32) | k0;
    const unsigned long long subseq = (c3 << 32) | c2;
    const unsigned long long offset = ((c1 << 32) | c0) * 4ULL;
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    unsigned int r0 = e(), r1 = e(), r2 = e(), r3 = e();
    std::printf("%u %u %u %u\n", r0, r1, r2, r3);
  }
  return 0;
}
