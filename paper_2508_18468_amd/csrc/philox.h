// Philox4x64-10 counter-based random numbers, device side.
//
// From the published definition (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): two 64x64->128-bit multiplies per
// round with multipliers M0, M1; the two key words are bumped by the Weyl
// constants W0, W1 between rounds; ten rounds.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mfq {

struct u64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1,
                                               uint64_t c2, uint64_t c3) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return u64x4{{c0, c1, c2, c3}};
}

// Open-interval uniform: ((x >> 12) + 0.5) * 2^-52, every value exact.
__device__ __forceinline__ double u01(uint64_t x) {
  return ((double)(x >> 12) + 0.5) * 0x1.0p-52;
}

enum { PURPOSE_PROJECTIVE = 0, PURPOSE_HOMODYNE = 1, PURPOSE_CONTINUOUS = 2 };

}  // namespace mfq
