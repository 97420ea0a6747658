// philox.h -- device Philox4x32-10 counter-based generator (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and the
// coordinate draw of the adaptive estimator (Section 4: coordinates drawn
// uniformly from [m]).
//
// The draw for sample t of point i under seed s is output (t mod 4) of
// Philox4x32-10 with key (s lo, s hi) and counter (t/4, 0, i, 0) -- the same
// stream as rocRAND's philox engine with subsequence i and offset t.  A
// 32-bit draw r maps to the coordinate floor(r m / 2^32).  When one
// coordinate sequence serves every point (the estimator of Section 4 is
// written over indices j_1, j_2, ... that need not depend on the point), the
// counter is (t/4, 0, 0, 2) instead.
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

// Sampling without replacement (Section 4 footnote): sample t < m of point i
// is pi(t) for a permutation pi of [0, m) keyed by (seed, i): a four-round
// Feistel network on 2h bits (h = max(1, ceil(ceil(log2 m) / 2)), halves of h
// bits, (L, R) -> (R, L xor F(k_r, R)), F(k, v) = lowbias32(v xor k) mod
// 2^h), with round keys Philox4x32-10(seed, counter (0, 0, i, 1)) and cycle
// walking into [0, m) (Black & Rogaway 2002).  lowbias32 is C. Wellons'
// 32-bit integer hash (hash-prospector).
struct PermKey {
  uint32_t k[4];
};

// Counter words (c2, c3) of point i's draws: (i, 0) per point, with the
// permutation's round keys at (i, 1); one sequence shared by all points
// uses (0, 2) and (0, 3).
__device__ __forceinline__ uint32_t draw_c2(uint32_t i, bool shared) { return shared ? 0u : i; }
__device__ __forceinline__ uint32_t draw_c3(bool shared, bool perm) { return (shared ? 2u : 0u) | (perm ? 1u : 0u); }

__device__ __forceinline__ PermKey perm_key(uint32_t c2, uint32_t c3, uint32_t s0, uint32_t s1) {
  const P4 r = philox10(0u, 0u, c2, c3, s0, s1);
  return PermKey{{r.x, r.y, r.z, r.w}};
}

__device__ __forceinline__ int perm_half_bits(uint32_t m) {
  const int bits = m <= 1u ? 0 : 32 - __clz(m - 1u);  // ceil(log2 m)
  const int h = (bits + 1) / 2;
  return h < 1 ? 1 : h;
}

__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint32_t perm_coord(uint32_t t, uint32_t m, int h, const PermKey &pk) {
  const uint32_t mask = (1u << h) - 1u;  // h <= 16 for m < 2^32
  uint32_t x = t;
  do {
    uint32_t L = (x >> h) & mask, R = x & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t nr = L ^ (lowbias32(R ^ pk.k[r]) & mask);
      L = R;
      R = nr;
    }
    x = (L << h) | R;
  } while (x >= m);
  return x;
}

// The four coordinates of draw block b (samples 4b .. 4b + 3) of the
// sequence with counter words (c2, c3) (draw_c2 / draw_c3).
__device__ __forceinline__ void draw_block(uint32_t b, uint32_t c2, uint32_t c3, uint32_t s0, uint32_t s1, uint32_t m,
                                           bool norepl, int h, const PermKey &pk, uint32_t (&js)[4]) {
  if (norepl) {
#pragma unroll
    for (int e = 0; e < 4; ++e) js[e] = perm_coord(4u * b + (uint32_t)e, m, h, pk);
  } else {
    const P4 r = philox10(b, 0u, c2, c3, s0, s1);
    js[0] = coord_of(r.x, m);
    js[1] = coord_of(r.y, m);
    js[2] = coord_of(r.z, m);
    js[3] = coord_of(r.w, m);
  }
}

}  // namespace knn
