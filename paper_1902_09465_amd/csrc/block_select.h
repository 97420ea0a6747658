// block_select.h -- exact order statistics of 64-bit keys inside one
// workgroup, by most-significant-digit radix selection with an LDS
// histogram (8-bit digits).  Only values matter for the thresholds of the
// adaptive rule, so keys are selected with multiplicity; where an index
// tie-break is needed the caller runs a second selection on the indices of
// the boundary key.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "knn_prof.h"

namespace knn {

constexpr int kWave = 64;

struct SelScratch {
  uint32_t hist[256];
  int32_t res[4];
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Work item of this block for a 1-D grid of 8 * ceil(nwork / 8) blocks.
// Consecutive blocks are dispatched round-robin over the 8 XCDs, each with
// its own L2; this mapping gives every XCD one contiguous range of work
// items instead, so items that read the same lines (neighbours in the work
// order) run on the same XCD at nearly the same time.  Items >= nwork are
// padding (the block has nothing to do).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_work_item(int64_t nwork) {
  const int64_t per = (nwork + kXcds - 1) / kXcds;
  return (int64_t)(blockIdx.x % kXcds) * per + (int64_t)(blockIdx.x / kXcds);
}
inline int64_t xcd_grid(int64_t nwork) { return (nwork + kXcds - 1) / kXcds * kXcds; }

// One wave: find the bucket b where the running count over hist[0..255]
// first reaches r (1-based); res[0] = b, res[1] = count in buckets < b.
__device__ __forceinline__ void scan_find_bucket(SelScratch &s, int r) {
  const int l = lane_id();
  const uint32_t c0 = s.hist[4 * l], c1 = s.hist[4 * l + 1], c2 = s.hist[4 * l + 2],
                 c3 = s.hist[4 * l + 3];
  const int tot = (int)(c0 + c1 + c2 + c3);
  int incl = tot;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = __shfl_up(incl, d);
    if (l >= d) incl += t;
  }
  const int excl = incl - tot;
  if (excl < r && r <= incl) {
    int cum = excl;
    int b;
    if (cum + (int)c0 >= r) {
      b = 4 * l;
    } else {
      cum += (int)c0;
      if (cum + (int)c1 >= r) {
        b = 4 * l + 1;
      } else {
        cum += (int)c1;
        if (cum + (int)c2 >= r) {
          b = 4 * l + 2;
        } else {
          cum += (int)c2;
          b = 4 * l + 3;
        }
      }
    }
    s.res[0] = b;
    s.res[1] = cum;
  }
}

// rank-th smallest (1-based, with multiplicity) of the keys held in
// registers by the block (E per thread; pad unused entries with
// UINT64_MAX and count them).  *less = number of keys strictly smaller.
template <int NT, int E>
__device__ uint64_t block_kth_regs(const uint64_t (&key)[E], int rank, SelScratch &s, int *less) {
  uint64_t prefix = 0, mask = 0;
  int r = rank, lt = 0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += NT) s.hist[b] = 0;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
      if ((key[e] & mask) == prefix) atomicAdd(&s.hist[(uint32_t)(key[e] >> shift) & 255u], 1u);
    __syncthreads();
    if (threadIdx.x < kWave) scan_find_bucket(s, r);
    __syncthreads();
    const int b = s.res[0], before = s.res[1];
    r -= before;
    lt += before;
    prefix |= (uint64_t)b << shift;
    mask |= 0xFFull << shift;
    __syncthreads();
  }
  *less = lt;
  return prefix;
}

// Same over a generated sequence: getkey(p) for p in [0, N), re-evaluated on
// each of the 8 passes (the caller pads nothing; rank <= N).
template <int NT, typename GetKey>
__device__ uint64_t block_kth_gen(int64_t N, GetKey getkey, int rank, SelScratch &s, int *less) {
  uint64_t prefix = 0, mask = 0;
  int r = rank, lt = 0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += NT) s.hist[b] = 0;
    __syncthreads();
    for (int64_t p = threadIdx.x; p < N; p += NT) {
      const uint64_t k = getkey(p);
      if ((k & mask) == prefix) atomicAdd(&s.hist[(uint32_t)(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kWave) scan_find_bucket(s, r);
    __syncthreads();
    const int b = s.res[0], before = s.res[1];
    r -= before;
    lt += before;
    prefix |= (uint64_t)b << shift;
    mask |= 0xFFull << shift;
    __syncthreads();
  }
  *less = lt;
  return prefix;
}

// rank-th smallest 32-bit value among getval(p) for which keep(p) holds.
template <int NT, typename GetVal, typename Keep>
__device__ uint32_t block_kth_u32_gen(int64_t N, GetVal getval, Keep keep, int rank, SelScratch &s) {
  uint32_t prefix = 0, mask = 0;
  int r = rank;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += NT) s.hist[b] = 0;
    __syncthreads();
    for (int64_t p = threadIdx.x; p < N; p += NT) {
      if (!keep(p)) continue;
      const uint32_t v = getval(p);
      if ((v & mask) == prefix) atomicAdd(&s.hist[(v >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kWave) scan_find_bucket(s, r);
    __syncthreads();
    r -= s.res[1];
    prefix |= (uint32_t)s.res[0] << shift;
    mask |= 0xFFu << shift;
    __syncthreads();
  }
  return prefix;
}

// Lane l receives lane (l ^ j)'s value, for a j that is a constant after
// unrolling.  Every lane of the wave must be active.  No exchange goes
// through the LDS unit: within a quad and a 16-lane row they are DPP moves
// (xor 4 as the half-row mirror, lane i to 7 - i, then the quad reversal,
// i to i ^ 3: together i to i ^ 4), across rows the gfx950 lane swaps (the
// swap of a register with itself leaves the partner rows in one of its two
// results).
__device__ __forceinline__ uint32_t lane_xor_u32(uint32_t v, int j) {
  switch (j) {
    case 1:
      return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    case 2:
      return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    case 4: {
      const int t = __builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true);  // row_half_mirror
      return (uint32_t)__builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, true);      // quad_perm [3,2,1,0]
    }
    case 8:
      return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);  // row_ror:8 (16-lane rows)
    case 16: {
      // rows (0,1) and (2,3) swapped: the first result holds row r ^ 1 in rows 1 and 3, the second in rows 0 and 2
      const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
      return (__lane_id() & 16) ? r[0] : r[1];
    }
    default: {  // 32: halves swapped, likewise
      const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
      return (__lane_id() & 32) ? r[0] : r[1];
    }
  }
}
__device__ __forceinline__ uint64_t lane_xor_u64(uint64_t v, int j) {
  const uint32_t lo = lane_xor_u32((uint32_t)v, j), hi = lane_xor_u32((uint32_t)(v >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of one 64-bit key per lane across the wave (ascending with
// the lane index), by exchanges between lanes: 21 compare-exchange steps.
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint64_t o = lane_xor_u64(v, j);
      const bool keep_min = (((l & j) == 0) == ((l & k) == 0));
      v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
    }
  }
  return v;
}

// The same network on one 32-bit key per lane (one exchange per step).
__device__ __forceinline__ uint32_t wave_sort_u32(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t o = lane_xor_u32(v, j);
      const bool keep_min = (((l & j) == 0) == ((l & k) == 0));
      v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
    }
  }
  return v;
}

// This block's copy of the measurement counters (kProfCopies copies,
// kProfStride words apart).
__device__ __forceinline__ uint64_t *prof_copy(uint64_t *c) {
  return c + ((blockIdx.x + blockIdx.y * gridDim.x) % (unsigned)kProfCopies) * (unsigned)kProfStride;
}

// Adds each lane's v to *ctr with one atomic per wave (every lane of the
// wave must be active): a per-lane atomic on one address serialises at L2.
__device__ __forceinline__ void wave_count_add(uint64_t *ctr, uint64_t v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
    v += ((uint64_t)hi << 32) | lo;
  }
  if (lane_id() == 0 && v != 0) atomicAdd(ctr, v);
}

// Lane l receives lane (63 - l)'s value: the row mirror (l ^ 15 within a
// 16-lane row, a DPP move), then rows swapped by xor 16 and xor 32.
__device__ __forceinline__ uint32_t lane_rev_u32(uint32_t v) {
  const uint32_t m = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true);  // row_mirror
  return lane_xor_u32(lane_xor_u32(m, 16), 32);
}
__device__ __forceinline__ uint64_t wave_bcast_rev_u64(uint64_t v) {
  return ((uint64_t)lane_rev_u32((uint32_t)(v >> 32)) << 32) | lane_rev_u32((uint32_t)v);
}

// Every lane receives lane src's value (src the same in every lane).
__device__ __forceinline__ uint64_t wave_bcast_u64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// In-LDS bitonic sort of (key, idx) pairs ascending by (key, idx); len is a
// power of two; the whole block takes part.
template <int NT>
__device__ void block_bitonic_sort(uint64_t *key, int32_t *idx, int len) {
  for (int size = 2; size <= len; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < (len >> 1); t += NT) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const uint64_t ka = key[lo], kb = key[hi];
        const int32_t ia = idx[lo], ib = idx[hi];
        const bool a_gt_b = (ka > kb) || (ka == kb && ia > ib);
        if (a_gt_b == up) {
          key[lo] = kb;
          key[hi] = ka;
          idx[lo] = ib;
          idx[hi] = ia;
        }
      }
    }
  }
  __syncthreads();
}

// Running k smallest of unique 64-bit keys held by one wave in `list`
// (k <= KC entries, LDS), with tau = the current maximum: each candidate
// below tau replaces the maximum, which is then recomputed.  c0, c1 are this
// lane's two candidates.
template <int KC>
__device__ __forceinline__ void topk_insert(uint64_t *list, int k, uint64_t &tau, uint64_t c0, uint64_t c1) {
  const int lane = lane_id();
  bool p0 = c0 < tau, p1 = c1 < tau;
  uint64_t act = __ballot(p0 || p1);
  while (act) {
    const int src = __ffsll((long long)act) - 1;
    const bool use0 = __shfl((int)p0, src) != 0;
    const uint64_t cs = use0 ? c0 : c1;
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)cs, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(cs >> 32), src);
    const uint64_t cand = ((uint64_t)hi << 32) | lo;
    if (lane == src) {
      if (use0) p0 = false;
      else p1 = false;
    }
    // replace the slot holding tau (keys are unique)
#pragma unroll
    for (int e = 0; e < KC / 64; ++e) {
      const int j = e * 64 + lane;
      if (j < k && list[j] == tau) list[j] = cand;
    }
    // new maximum
    uint64_t mx = 0;
#pragma unroll
    for (int e = 0; e < KC / 64; ++e) {
      const int j = e * 64 + lane;
      if (j < k) mx = list[j] > mx ? list[j] : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t l2 = (uint32_t)__shfl_xor((int)(uint32_t)mx, o);
      const uint32_t h2 = (uint32_t)__shfl_xor((int)(uint32_t)(mx >> 32), o);
      const uint64_t v = ((uint64_t)h2 << 32) | l2;
      mx = v > mx ? v : mx;
    }
    tau = mx;
    p0 = p0 && (c0 < tau);
    p1 = p1 && (c1 < tau);
    act = __ballot(p0 || p1);
  }
}

// list: sorted ascending over the lanes; cand: one key per lane (PAD = none).
// Returns the 64 smallest of both, sorted ascending over the lanes.
__device__ __forceinline__ uint64_t merge_sorted64(uint64_t list, uint64_t cand) {
  const int lane = lane_id();
  uint64_t c = wave_sort_u64(cand);
  c = wave_bcast_rev_u64(c);  // descending
  uint64_t v = list < c ? list : c;
#pragma unroll
  for (int j = kWave / 2; j > 0; j >>= 1) {
    const uint64_t o = lane_xor_u64(v, j);
    v = ((lane & j) == 0) ? (o < v ? o : v) : (o > v ? o : v);
  }
  return v;
}

}  // namespace knn
