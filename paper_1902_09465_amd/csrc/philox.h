// philox.h -- device Philox4x32-10 counter-based generator (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and the
// coordinate draw of the adaptive estimator (Section 4: coordinates drawn
// uniformly from [m]).
//
// The draw for sample t of point i under seed s is output (t mod 4) of
// Philox4x32-10 with key (s lo, s hi) and counter (t/4, 0, i, 0) -- the same
// stream as rocRAND's philox engine with subsequence i and offset t.  A
// 32-bit draw r maps to the coordinate floor(r m / 2^32).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knn {

struct P4 {
  uint32_t x, y, z, w;
};

// Ten rounds.  The key schedule (k0 + r W0, k1 + r W1) is uniform across a
// wave when the seed is, so the compiler keeps it in scalar registers.
__device__ __forceinline__ P4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c0;
    const uint64_t p1 = (uint64_t)M1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += W0;
    k1 += W1;
  }
  return P4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t coord_of(uint32_t r, uint32_t m) {
  return __umulhi(r, m);
}

}  // namespace knn
