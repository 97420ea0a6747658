// k_adaptive.hip -- device side of the round-synchronous adaptive k-NN
// (Algorithm 1 of LeJeune, Baraniuk, Heckel, AISTATS 2019, one round at a
// time for every in-flight query "slot").
//
// One step advances every running slot by one round:
//   k_sample          draw and accumulate the round's samples (Section 4
//                     estimator), or the exact distance in the exact round
//   k_cand_partial/   optional: make the c_exact undecided points with the
//   k_cand_merge      smallest estimate exact
//   k_select_partial  per chunk of the kept set P: the k smallest upper and
//                     k+1 smallest lower bounds (values)
//   k_select_merge    U, L1, L2 for the slot (eq. d_ind in round form)
//   k_decide          discard / accept / keep, compacting the undecided list
//   k_finish          stop rule, output, next round, admission of new queries
// Query-lane batches that keep their running sums point-major use
// k_sample_ql_u8 (or the exact round as one tiled pass), k_select_pm,
// k_select_merge_pm and k_decide_pm instead, with the sets held as flags.
// All decisions use the same IEEE double expressions as the CPU oracle
// (compiled without FMA contraction); sums are integers, so the result does
// not depend on launch shape, chunking or atomic order.
#include <algorithm>
#include <cstdlib>

#include "block_select.h"
#include "knn_internal.h"
#include "philox.h"
#include "knn_prof.h"

namespace knn {

constexpr int NT = 256;

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int64_t shfl_i64(int64_t v, int src) {
  const int lo = __shfl((int)(uint32_t)v, src);
  const int hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int64_t shfl_xor_i64(int64_t v, int mask) {
  const int lo = __shfl_xor((int)(uint32_t)v, mask);
  const int hi = __shfl_xor((int)(uint32_t)((uint64_t)v >> 32), mask);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// floor(v * 2^F) for a finite v >= 0 with v 2^F < 2^64 (the f32
// fixed-point sample; every sample is below 2^61 by the choice of F), in two
// 32-bit halves from fp32 steps that are all exact: y = v 2^(F-32) is a
// power-of-two scaling, hi = floor(y), and lo = floor(fract(y) 2^32), where
// fract(y) = y - floor(y) is a float again.  Where y would be subnormal,
// v 2^F < 2^-94 and both halves are 0.  No branches: eight VALU operations
// per sample with the subtraction, the square and the 64-bit add.
__device__ __forceinline__ int64_t fixed_of(float v, int F) {
  const float y = __builtin_amdgcn_ldexpf(v, F - 32);
  const uint32_t hi = (uint32_t)y;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ldexpf(__builtin_amdgcn_fractf(y), 32);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One sample of coordinate j: (x_ij - x_j)^2, or |x_ij - x_j| for the l1
// distance (f32: in fixed point, floor(v 2^F)).
template <int DT, int MET>
__device__ __forceinline__ int64_t sample_val(const uint8_t *__restrict__ row,
                                              const uint8_t *__restrict__ q, uint32_t j, int F) {
  if constexpr (DT == KNN_U8) {
    const int d = (int)row[j] - (int)q[j];
    if constexpr (MET == KNN_METRIC_L1) return (int64_t)(d < 0 ? -d : d);
    return (int64_t)__mul24(d, d);  // |d| < 2^8: the full-rate 24-bit multiply is exact
  } else {
    const float d = reinterpret_cast<const float *>(row)[j] - reinterpret_cast<const float *>(q)[j];
    if constexpr (MET == KNN_METRIC_L1) return fixed_of(fabsf(d), F);
    return fixed_of(d * d, F);
  }
}

struct SlotArrays {
  int64_t *S;
  uint8_t *fl, *ri;
  int32_t *act, *xa;      // current halves
  int32_t *act_n, *xa_n;  // next halves
  int32_t *acc;
};

__device__ __forceinline__ SlotArrays slot_arrays(const Bufs &B, int64_t n, int s, int par) {
  SlotArrays a;
  a.S = B.S + (int64_t)s * n;
  a.fl = B.fl + (int64_t)s * n;
  a.ri = B.ri + (int64_t)s * n;
  int32_t *act = B.act + (int64_t)s * 2 * n;
  int32_t *xa = B.xa + (int64_t)s * 2 * n;
  a.act = act + (int64_t)par * n;
  a.act_n = act + (int64_t)(par ^ 1) * n;
  a.xa = xa + (int64_t)par * n;
  a.xa_n = xa + (int64_t)(par ^ 1) * n;
  a.acc = B.acc + (int64_t)s * n;
  return a;
}

// Estimate and width of point i (Section 4): d^ = S / (T W), alpha(T); an
// exact point has T = m and width 0 (Algorithm 1).
__device__ __forceinline__ void point_bounds(const Slot *sl, int64_t m, int64_t S, uint8_t f,
                                             uint8_t r, double &d, double &a) {
  if (f & FL_EXACT) {
    d = (double)S / ((double)m * sl->W);
    a = 0.0;
  } else {
    d = (double)S / ((double)sl->T[r] * sl->W);
    a = sl->alpha[r];
  }
}

// p-th element of the kept set P = [act | xa | acc] (identity in round 0).
// Dense slots of point-major batches (implicit 2) are never enumerated this
// way: their kernels read the sets from the flags.
__device__ __forceinline__ int32_t elem_P(const Slot *sl, const SlotArrays &a, int64_t p) {
  if (sl->implicit) return (int32_t)p;
  if (p < sl->n_act) return a.act[p];
  p -= sl->n_act;
  if (p < sl->n_xa) return a.xa[p];
  return a.acc[p - sl->n_xa];
}

// p-th element of the undecided set A = [act | xa] (identity in round 0).
__device__ __forceinline__ int32_t elem_A(const Slot *sl, const SlotArrays &a, int64_t p) {
  if (sl->implicit) return (int32_t)p;
  if (p < sl->n_act) return a.act[p];
  return a.xa[p - sl->n_act];
}

__device__ __forceinline__ int64_t size_P(const Slot *sl, int64_t n) {
  return sl->implicit ? n : (int64_t)sl->n_act + sl->n_xa + sl->n_acc;
}
__device__ __forceinline__ int64_t size_A(const Slot *sl, int64_t n) {
  return sl->implicit ? n : (int64_t)sl->n_act + sl->n_xa;
}

// Exact sum over all m coordinates of point i by the whole block
// (rare paths: candidate-exact and oversized finalisation).
template <int DT, int BT>
__device__ int64_t block_exact_sum(const uint8_t *X, int64_t m, int32_t i, const uint8_t *q, int F, int met,
                                   int64_t *red) {
  const int elem = DT == KNN_U8 ? 1 : 4;
  const uint8_t *row = X + (int64_t)i * m * elem;
  int64_t acc = 0;
  if (met == KNN_METRIC_L1) {
    for (int64_t j = threadIdx.x; j < m; j += BT) acc += sample_val<DT, KNN_METRIC_L1>(row, q, (uint32_t)j, F);
  } else {
    for (int64_t j = threadIdx.x; j < m; j += BT) acc += sample_val<DT, KNN_METRIC_L2>(row, q, (uint32_t)j, F);
  }
  for (int o = kWave / 2; o > 0; o >>= 1) acc += shfl_xor_i64(acc, o);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  int64_t tot = 0;
  for (int w = 0; w < BT / kWave; ++w) tot += red[w];
  __syncthreads();
  return tot;
}

// ---------------------------------------------------------------- f32 prep

// Per query: value range of query and points -> W = R' 2^F with
// R' = (hi - lo)^2 (1 + 2^-20) (l1: (hi - lo)(1 + 2^-20)),
// F = 61 - ceil(log2 m) - ceil(log2 R').
__device__ __forceinline__ int ceil_log2_pos(double x) {
  uint64_t b;
  __builtin_memcpy(&b, &x, 8);
  const int fe = (int)((b >> 52) & 0x7FF) - 1022;  // x = f 2^fe, f in [0.5, 1)
  return (b & 0xFFFFFFFFFFFFFull) == 0 ? fe - 1 : fe;
}
__device__ __forceinline__ double pow2_d(int e) {
  const uint64_t b = (uint64_t)(e + 1023) << 52;
  double x;
  __builtin_memcpy(&x, &b, 8);
  return x;
}

__global__ __launch_bounds__(NT) void k_prep_f32(QDesc *qd, int32_t nq, int64_t n, int64_t m,
                                                 double db_lo, double db_hi, int32_t metric) {
  const int qi = blockIdx.x;
  if (qi >= nq) return;
  const float *q = reinterpret_cast<const float *>(qd[qi].q);
  float lo = INFINITY, hi = -INFINITY;
  for (int64_t j = threadIdx.x; j < m; j += NT) {
    lo = fminf(lo, q[j]);
    hi = fmaxf(hi, q[j]);
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o));
    hi = fmaxf(hi, __shfl_xor(hi, o));
  }
  __shared__ float slo[NT / kWave], shi[NT / kWave];
  if (lane_id() == 0) {
    slo[threadIdx.x / kWave] = lo;
    shi[threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double l = db_lo, h = db_hi;
    for (int w = 0; w < NT / kWave; ++w) {
      if ((double)slo[w] < l) l = (double)slo[w];
      if ((double)shi[w] > h) h = (double)shi[w];
    }
    const double span = h - l;
    if (!(span > 0.0)) {
      qd[qi].trivial = 1;
      qd[qi].W = 0.0;
      qd[qi].F = 0;
    } else {
      // the largest sample, (hi - lo)^2 or (l1) hi - lo, with room for fp32 rounding
      const double Rp = (metric == KNN_METRIC_L1 ? span : span * span) * (1.0 + 0x1p-20);
      const int F = 61 - ceil_log2_pos((double)m) - ceil_log2_pos(Rp);
      qd[qi].F = F;
      qd[qi].W = Rp * pow2_d(F);
      if (qd[qi].kh >= n) qd[qi].trivial = 1;
    }
  }
}

// ---------------------------------------------------------------- sample

// Round `cur` of every running slot: samples t in [T[cur-1], T[cur]) of each
// point of the sampled list, LPP lanes per point (each lane takes every
// LPP-th block of four draws); or, in the exact round, the exact distance,
// one wave per point with coalesced row reads.
template <int DT, int MET, bool QLDS, int BT = NT>
__device__ void sample_slot_chunk(const Slot *sl, int s, int64_t chunk, const uint8_t *__restrict__ X,
                                  const Bufs &B, const Geometry &G, uint8_t *smem) {
  const int64_t n = G.n, m = G.m;
  const int implicit = sl->implicit;
  const int64_t nlist = implicit ? n : sl->n_act;
  const int64_t base = chunk * G.ch_sample;
  if (base >= nlist) return;
  const int64_t end = min(nlist, base + (int64_t)G.ch_sample);
  constexpr int elem = DT == KNN_U8 ? 1 : 4;
  const uint8_t *qg = reinterpret_cast<const uint8_t *>(sl->q);
  if constexpr (QLDS) {
    const int64_t qb = m * elem;
    if ((qb & 3) == 0 && (((uintptr_t)qg) & 3) == 0) {
      for (int64_t w = threadIdx.x; w < qb / 4; w += BT)
        reinterpret_cast<uint32_t *>(smem)[w] = reinterpret_cast<const uint32_t *>(qg)[w];
    } else {
      for (int64_t w = threadIdx.x; w < qb; w += BT) smem[w] = qg[w];
    }
    __syncthreads();
  }
  const uint8_t *q = QLDS ? smem : qg;
  const int cur = sl->cur;
  const int F = sl->F;
  const SlotArrays a = slot_arrays(B, n, s, sl->par);
  if (G.prof && threadIdx.x == 0) {
    // algorithmic work of this block: per point the sampled values, the
    // running sum (read + write), the list entry and the round index
    const uint64_t pts = (uint64_t)(end - base);
    if (cur >= sl->R) {
      atomicAdd(&prof_copy(G.prof)[0], pts * (uint64_t)(m * elem + 14));
      atomicAdd(&prof_copy(G.prof)[2], pts * (uint64_t)m);
    } else {
      const uint64_t B_r = (uint64_t)(sl->T[cur] - (cur ? sl->T[cur - 1] : 0));
      atomicAdd(&prof_copy(G.prof)[0], pts * (B_r * elem + 21));
      atomicAdd(&prof_copy(G.prof)[1], pts * B_r);
      atomicAdd(&prof_copy(G.prof)[3], pts * B_r);  // every sample is its own draw here
    }
  }
  if (cur >= sl->R) {
    // exact round
    const int wave = threadIdx.x / kWave, lane = lane_id();
    for (int64_t p = base + wave; p < end; p += BT / kWave) {
      const int32_t i = implicit ? (int32_t)p : a.act[p];
      const uint8_t *row = X + (int64_t)i * m * elem;
      int64_t acc = 0;
      if constexpr (DT == KNN_U8) {
        if ((m & 3) == 0) {
          const uint32_t *r4 = reinterpret_cast<const uint32_t *>(row);
          for (int64_t w = lane; w < m / 4; w += kWave) {
            const uint32_t xv = r4[w];
            const uint32_t qv = QLDS ? reinterpret_cast<const uint32_t *>(q)[w]
                                     : (uint32_t)q[4 * w] | ((uint32_t)q[4 * w + 1] << 8) |
                                           ((uint32_t)q[4 * w + 2] << 16) | ((uint32_t)q[4 * w + 3] << 24);
            if constexpr (MET == KNN_METRIC_L1) {
              // four absolute differences in one sum-of-absolute-differences
              acc += (int64_t)__builtin_amdgcn_sad_u8(xv, qv, 0u);
            } else {
              // four squared differences as x.x + q.q - 2 x.q (at most 4 * 255^2)
              const uint32_t sq = __builtin_amdgcn_udot4(xv, xv, 0u, false) +
                                  __builtin_amdgcn_udot4(qv, qv, 0u, false) - 2u * __builtin_amdgcn_udot4(xv, qv, 0u, false);
              acc += (int64_t)sq;
            }
          }
        } else {
          for (int64_t j = lane; j < m; j += kWave) acc += sample_val<DT, MET>(row, q, (uint32_t)j, F);
        }
      } else {
        for (int64_t j = lane; j < m; j += kWave) acc += sample_val<DT, MET>(row, q, (uint32_t)j, F);
      }
      for (int o = kWave / 2; o > 0; o >>= 1) acc += shfl_xor_i64(acc, o);
      if (lane == 0) {
        a.S[i] = acc;
        if (cur == 0) {
          a.fl[i] = FL_EXACT;
          a.ri[i] = 0;
        } else {
          a.fl[i] = a.fl[i] | FL_EXACT;
        }
      }
    }
    __syncthreads();  // smem (the staged query) may be reused by the caller
    return;
  }
  // sampled round
  const uint32_t t0 = cur ? (uint32_t)sl->T[cur - 1] : 0u;
  const uint32_t t1 = (uint32_t)sl->T[cur];
  const uint32_t blk0 = t0 >> 2, blk1 = t1 >> 2;
  const uint32_t k0 = (uint32_t)sl->seed, k1 = (uint32_t)(sl->seed >> 32);
  const uint32_t mm = (uint32_t)m;
  // lanes per point: enough that every lane draws at least one block of four
  // samples, up to a whole wave, so a wave's gathers hit one or a few rows
  int lpp = G.lpp;
  if (lpp <= 0) {
    const uint32_t nb = blk1 - blk0;
    lpp = 1;
    while (lpp < kWave && (uint32_t)(2 * lpp) <= nb) lpp <<= 1;
  }
  const int sub = threadIdx.x % lpp;
  const bool norepl = sl->norepl != 0, shared = sl->shared != 0;
  const int ph = perm_half_bits(mm);
  const uint32_t c3 = draw_c3(shared, false);
  for (int64_t p = base + threadIdx.x / lpp; p < end; p += BT / lpp) {
    const int32_t i = implicit ? (int32_t)p : a.act[p];
    const uint8_t *row = X + (int64_t)i * m * elem;
    const uint32_t c2 = draw_c2((uint32_t)i, shared);
    const PermKey pk = norepl ? perm_key(c2, draw_c3(shared, true), k0, k1) : PermKey{{0u, 0u, 0u, 0u}};
    int64_t acc = 0;
    for (uint32_t b = blk0 + sub; b < blk1; b += lpp) {
      uint32_t js[4];
      draw_block(b, c2, c3, k0, k1, mm, norepl, ph, pk, js);
#pragma unroll
      for (int e = 0; e < 4; ++e) acc += sample_val<DT, MET>(row, q, js[e], F);
    }
    for (int o = lpp / 2; o > 0; o >>= 1) acc += shfl_xor_i64(acc, o);
    if (sub == 0) {
      if (cur == 0) {
        a.S[i] = acc;
        a.fl[i] = 0;
      } else {
        a.S[i] += acc;
      }
      a.ri[i] = (uint8_t)cur;
    }
  }
  __syncthreads();  // smem (the staged query) may be reused by the caller
}


// The exact round of a lock-step fp32 batch as one tiled pass over (slots x
// points): per block 64 slots x 128 points, 32-coordinate slices of the
// query and point rows staged transposed in LDS, each thread 8 slots x 4
// points.  Every pair that the per-slot exact pass would make exact (flag 0,
// or every point in round 0) gets the same integer sum of the same
// fixed-point samples fixed_of(fl32(x - q)^2, F) (or |x - q| for l1), so the
// result is the same; the rows are read once per 64 slots instead of once
// per slot.
constexpr int XF_Q = 64, XF_P = 128, XF_K = 32;
// Columns [c0, c1) of rows of `stride` floats: the points X (or their copy
// gathered at a shared coordinate sequence) and the queries (the slots' own
// rows, or QS [slot][stride] of the gathered queries).  mode 0: the exact
// round -- the pairs' sums become these columns' sums and the pairs exact;
// mode 1: a sampled round -- added to the sums of the undecided sampled
// pairs (round 0: every pair, sums set), round index cur; mode 2: the exact
// round of sampling without replacement -- the columns not yet sampled are
// added and the pairs become exact.  Only slots at round `cur` take part.
template <int MET>
__global__ __launch_bounds__(NT) void k_exact_f32_tile(const Slot *__restrict__ slots, const float *__restrict__ X,
                                                       int64_t stride, int64_t c0, int64_t c1,
                                                       const float *__restrict__ QS, int32_t mode, int32_t cur,
                                                       Bufs B, Geometry G) {
  __shared__ __align__(16) float qs[XF_K][XF_Q + 4];  // (rows of 68 and 132 floats: 16-byte aligned)
  __shared__ __align__(16) float xs[XF_K][XF_P + 4];
  __shared__ const float *qrow[XF_Q];
  __shared__ int qF[XF_Q];
  __shared__ uint8_t take[XF_Q], impl[XF_Q];
  __shared__ int any;
  const int64_t n = G.n;
  const int ns = G.nslots;
  const int64_t nqt = (ns + XF_Q - 1) / XF_Q, nwork = nqt * ((n + XF_P - 1) / XF_P);
  const int64_t w = xcd_work_item(nwork);
  if (w >= nwork) return;
  const int64_t p0 = (w / nqt) * XF_P;  // query tiles of one point tile back to back (rows from L2)
  const int q0 = (int)(w % nqt) * XF_Q;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (threadIdx.x < XF_Q) {
    const int s = q0 + threadIdx.x;
    // (cur < 0: every slot at its exact round)
    const bool t = s < ns && slots[s].state == 1 && (cur < 0 ? slots[s].cur >= slots[s].R : slots[s].cur == cur);
    take[threadIdx.x] = t ? 1 : 0;
    impl[threadIdx.x] = (t && slots[s].implicit) ? 1 : 0;
    qrow[threadIdx.x] = !t ? nullptr : (QS ? QS + (int64_t)s * stride : reinterpret_cast<const float *>(slots[s].q));
    qF[threadIdx.x] = t ? slots[s].F : 0;
    if (t) any = 1;
  }
  __syncthreads();
  if (!any) return;  // (block-uniform) no slot of this query tile is at this round
  const int qg = threadIdx.x % 8, pg = threadIdx.x / 8;  // slots 8 qg .. 8 qg + 7, points 4 pg .. 4 pg + 3
  int64_t acc[8][4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  int F[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) F[a] = qF[8 * qg + a];
  for (int64_t k0 = c0; k0 < c1; k0 += XF_K) {
    // stage the slice transposed: [coordinate][slot] and [coordinate][point]
    for (int e = threadIdx.x; e < XF_Q * XF_K; e += NT) {
      const int ql = e / XF_K, kk = e % XF_K;
      const float *qr = qrow[ql];
      qs[kk][ql] = (qr && k0 + kk < c1) ? qr[k0 + kk] : 0.0f;
    }
    for (int e = threadIdx.x; e < XF_P * XF_K; e += NT) {
      const int pl = e / XF_K, kk = e % XF_K;
      const int64_t i = p0 + pl;
      xs[kk][pl] = (i < n && k0 + kk < c1) ? X[i * stride + k0 + kk] : 0.0f;
    }
    __syncthreads();
    const int kend = (int)min((int64_t)XF_K, c1 - k0);
    for (int kk = 0; kk < kend; ++kk) {
      const float4 qa = *reinterpret_cast<const float4 *>(&qs[kk][8 * qg]);
      const float4 qb = *reinterpret_cast<const float4 *>(&qs[kk][8 * qg + 4]);
      const float4 xv = *reinterpret_cast<const float4 *>(&xs[kk][4 * pg]);
      const float qv[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
      const float xx[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const float d = xx[b] - qv[a];
          acc[a][b] += MET == KNN_METRIC_L1 ? fixed_of(fabsf(d), F[a]) : fixed_of(d * d, F[a]);
        }
    }
    __syncthreads();
  }
  uint64_t my_pairs = 0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ql = 8 * qg + a;
    if (!take[ql]) continue;
    const int s = q0 + ql;
    const SlotArrays sa = slot_arrays(B, n, s, slots[s].par);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t i = p0 + 4 * pg + b;
      if (i >= n) continue;
      if (!impl[ql] && sa.fl[i] != 0) continue;  // only undecided sampled pairs
      if (mode == 1) {  // a sampled round
        if (impl[ql]) {
          sa.S[i] = acc[a][b];
          sa.fl[i] = 0;
        } else {
          sa.S[i] += acc[a][b];
        }
        sa.ri[i] = (uint8_t)cur;
      } else {
        sa.S[i] = (mode == 2 && !impl[ql]) ? sa.S[i] + acc[a][b] : acc[a][b];
        sa.fl[i] = FL_EXACT;
        if (impl[ql]) sa.ri[i] = 0;
      }
      ++my_pairs;
    }
  }
  if (G.prof) {  // whole waves reach this point
    const uint64_t cols = (uint64_t)(c1 - c0);
    wave_count_add(&prof_copy(G.prof)[mode == 1 ? 1 : 2], my_pairs * cols);
  }
}

template <int DT, int MET, bool QLDS>
__global__ __launch_bounds__(NT) void k_sample(Slot *__restrict__ slots, const uint8_t *__restrict__ X,
                                               Bufs B, Geometry G) {
  // slot-fastest grid: blocks that run together cover the same points for
  // many queries, so the point rows they gather stay in L2
  const int s = blockIdx.x;
  const Slot *sl = &slots[s];
  if (sl->state != 1) return;
  if (G.flagsets && sl->implicit != 0) return;  // a dense slot of a point-major batch
  extern __shared__ __align__(16) uint8_t smem[];
  // chunks blockIdx.y, blockIdx.y + gridDim.y, ... of the slot's list (a
  // grid narrower than the list is sized for the lists expected)
  const int64_t nlist = sl->implicit ? G.n : sl->n_act;
  for (int64_t c = blockIdx.y; c * G.ch_sample < nlist; c += gridDim.y) {
    sample_slot_chunk<DT, MET, QLDS>(sl, s, c, X, B, G, smem);
    __syncthreads();  // the next chunk restages the block's LDS
  }
}

// ---------------------------------------------------------------- grouped sample (u8)

// Sixteen slots that share the seed and the round draw the same coordinates
// for a point (the draw depends on (seed, point, sample) only), so one block
// serves all of them: one Philox draw and one gather of x_ij per sample,
// reused for every query of the group from a transposed query tile in LDS
// (one 16-byte read gives the sixteen query values at coordinate j).  In the
// exact round the group computes its sixteen rows of distances on the matrix
// cores: sum_j (x_ij - q_j)^2 = |x'|^2 + |q'|^2 - 2 x'.q' with x' = x - 128,
// q' = q - 128, exact in integers (int8 MFMA, int32 accumulation).  Groups
// whose slots differ in seed or round fall back to the per-slot path.
// Points are taken in index order; a slot's undecided-and-sampled points
// are exactly those with no flag set (all points in round 0).
constexpr int GRP = 16;
constexpr int GBT = 512;  // threads per block of the grouped kernel
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));

// Sums v[0..GRP) over the LPP lanes of a point (LPP a power of two <= 64)
// by halving exchanges: at each step a lane keeps one half of its values
// and receives the partner's copy of that half, so GRP values need about GRP
// shuffles in total instead of GRP log2(LPP).  Afterwards each lane holds the
// totals of GRP / min(LPP, GRP) consecutive slots; of the lanes holding the
// same slots (when LPP > GRP) the one with the low bits clear stores them.
// Everything is indexed with compile-time constants (no register spills).
template <int LPP>
__device__ __forceinline__ void reduce_store(uint32_t (&v)[GRP], int lane, uint32_t act, int g0, int64_t n,
                                             int32_t i, int cur, const Bufs &B) {
  constexpr int HALVINGS = (LPP >= GRP) ? 4 : (LPP == 8 ? 3 : LPP == 4 ? 2 : LPP == 2 ? 1 : 0);
  constexpr int NV = GRP >> HALVINGS;
  int base = 0;
#pragma unroll
  for (int st = 0; st < HALVINGS; ++st) {
    const int d = LPP >> (st + 1);
    const int half = GRP >> (st + 1);
    const bool up = (lane & d) != 0;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const uint32_t send = up ? v[k] : v[k + half];
      const uint32_t recv = (uint32_t)__shfl_xor((int)send, d);
      v[k] = (up ? v[k + half] : v[k]) + recv;
    }
    if (up) base += half;
  }
  int dup = 0;
#pragma unroll
  for (int d = (LPP >> (HALVINGS + 1)); d > 0; d >>= 1) {
    v[0] += (uint32_t)__shfl_xor((int)v[0], d);
    dup |= d;
  }
  if (lane & dup) return;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int g = base + k;
    if (!(act & (1u << g))) continue;
    const int64_t off = (int64_t)(g0 + g) * n + i;
    if (cur == 0) {
      B.S[off] = (int64_t)v[k];
      B.fl[off] = 0;
    } else {
      B.S[off] += (int64_t)v[k];
    }
    B.ri[off] = (uint8_t)cur;
  }
}

// Sum over this lane's share of the draws of one point, for the GRP queries
// of a group: blocks of four draws b = b_first, b_first + step, ... < blk1.
// (x - q)^2 over four draws is x.x - 2 x.q + q.q on four-byte vectors: the
// four draws' query bytes are transposed so that one dword holds one query's
// four values, and each product is one dot4.  `row` is the point's row, in
// global memory or staged in LDS; qT is the transposed query tile in LDS.
// The per-lane results are below 2^32 (at most m < 4096 draws of 255^2),
// so the modular combination at the end is exact.  For the l1 distance each
// query's four |x - q| are one v_sad_u8 on the same transposed dwords.
template <int MET>
__device__ __forceinline__ void point_sums(const uint8_t *row, const uint8_t *qT, uint32_t i, uint32_t b_first,
                                           uint32_t step, uint32_t blk1, uint32_t k0, uint32_t k1, uint32_t mm,
                                           bool norepl, bool shared, uint32_t (&acc)[GRP]) {
  uint32_t qq[GRP], xq[GRP], xx = 0;
#pragma unroll
  for (int g = 0; g < GRP; ++g) qq[g] = xq[g] = 0;
  const int ph = perm_half_bits(mm);
  const uint32_t c2 = draw_c2(i, shared), c3 = draw_c3(shared, false);
  const PermKey pk = norepl ? perm_key(c2, draw_c3(shared, true), k0, k1) : PermKey{{0u, 0u, 0u, 0u}};
  auto fetch = [&](uint32_t blk, uint32_t (&xv)[4], uint4 (&qv)[4]) {
    uint32_t js[4];
    draw_block(blk, c2, c3, k0, k1, mm, norepl, ph, pk, js);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xv[e] = row[js[e]];
      qv[e] = *reinterpret_cast<const uint4 *>(qT + (size_t)js[e] * GRP);
    }
  };
  auto consume = [&](const uint32_t (&xv)[4], const uint4 (&qv)[4]) {
    const uint32_t x4 = xv[0] | (xv[1] << 8) | (xv[2] << 16) | (xv[3] << 24);
    if constexpr (MET == KNN_METRIC_L2) xx = __builtin_amdgcn_udot4(x4, x4, xx, false);
    const uint32_t r[4][4] = {{qv[0].x, qv[1].x, qv[2].x, qv[3].x},
                              {qv[0].y, qv[1].y, qv[2].y, qv[3].y},
                              {qv[0].z, qv[1].z, qv[2].z, qv[3].z},
                              {qv[0].w, qv[1].w, qv[2].w, qv[3].w}};
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      // 4x4 byte transpose: c[u] = byte u of r[w][0..3]
      const uint32_t t0 = __builtin_amdgcn_perm(r[w][1], r[w][0], 0x05010400u);
      const uint32_t t1 = __builtin_amdgcn_perm(r[w][1], r[w][0], 0x07030602u);
      const uint32_t t2 = __builtin_amdgcn_perm(r[w][3], r[w][2], 0x05010400u);
      const uint32_t t3 = __builtin_amdgcn_perm(r[w][3], r[w][2], 0x07030602u);
      const uint32_t c[4] = {__builtin_amdgcn_perm(t2, t0, 0x05040100u), __builtin_amdgcn_perm(t2, t0, 0x07060302u),
                             __builtin_amdgcn_perm(t3, t1, 0x05040100u), __builtin_amdgcn_perm(t3, t1, 0x07060302u)};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if constexpr (MET == KNN_METRIC_L1) {
          xq[4 * w + u] = __builtin_amdgcn_sad_u8(x4, c[u], xq[4 * w + u]);
        } else {
          qq[4 * w + u] = __builtin_amdgcn_udot4(c[u], c[u], qq[4 * w + u], false);
          xq[4 * w + u] = __builtin_amdgcn_udot4(x4, c[u], xq[4 * w + u], false);
        }
      }
    }
  };
  // software pipelined over two register stages: the next block's draws,
  // gathers and LDS reads are in flight while one is summed
  uint32_t xa[4], xb[4];
  uint4 qa[4], qb[4];
  uint32_t b = b_first;
  if (b < blk1) fetch(b, xa, qa);
  while (b < blk1) {
    const uint32_t b1 = b + step;
    if (b1 < blk1) fetch(b1, xb, qb);
    consume(xa, qa);
    if (b1 >= blk1) break;
    const uint32_t b2 = b1 + step;
    if (b2 < blk1) fetch(b2, xa, qa);
    consume(xb, qb);
    b = b2;
  }
#pragma unroll
  for (int g = 0; g < GRP; ++g) acc[g] = MET == KNN_METRIC_L1 ? xq[g] : xx + qq[g] - 2u * xq[g];
}

// Flags of the point for the running slots of the group: bit g set when slot
// g0 + g still samples point i (in round 0 and with implicit lists: all).
__device__ __forceinline__ uint32_t group_active(const Bufs &B, int g0, int64_t n, int32_t i, uint32_t run,
                                                 int impl) {
  if (impl) return run;
  // sixteen independent loads in flight at once (run is uniform)
  const uint8_t *f = B.fl + (int64_t)g0 * n + i;
  uint32_t v[GRP];
#pragma unroll
  for (int g = 0; g < GRP; ++g) v[g] = (run & (1u << g)) ? (uint32_t)f[(int64_t)g * n] : 1u;
  uint32_t act = 0;
#pragma unroll
  for (int g = 0; g < GRP; ++g) act |= (v[g] == 0 ? 1u : 0u) << g;
  return act;
}

__device__ __forceinline__ void reduce_store_lpp(int lpp, uint32_t (&acc)[GRP], int lane, uint32_t act, int g0,
                                                 int64_t n, int32_t i, int cur, const Bufs &B) {
  switch (lpp) {
    case 1: reduce_store<1>(acc, lane, act, g0, n, i, cur, B); break;
    case 2: reduce_store<2>(acc, lane, act, g0, n, i, cur, B); break;
    case 4: reduce_store<4>(acc, lane, act, g0, n, i, cur, B); break;
    case 8: reduce_store<8>(acc, lane, act, g0, n, i, cur, B); break;
    case 16: reduce_store<16>(acc, lane, act, g0, n, i, cur, B); break;
    case 32: reduce_store<32>(acc, lane, act, g0, n, i, cur, B); break;
    default: reduce_store<64>(acc, lane, act, g0, n, i, cur, B); break;
  }
}

template <int MET>
__global__ __launch_bounds__(GBT) __attribute__((amdgpu_waves_per_eu(4))) void k_sample_grp_u8(Slot *__restrict__ slots, const uint8_t *__restrict__ X,
                                                      const int8_t *__restrict__ X8, const int32_t *__restrict__ xn,
                                                      int64_t mp, Bufs B, Geometry G) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ int s_mode, s_cur, s_impl, s_norepl, s_shared;
  __shared__ uint32_t s_run;
  __shared__ uint64_t s_seed;
  __shared__ uint32_t s_t0, s_t1;
  __shared__ int64_t s_qn[GBT / kWave];
  const int g0 = blockIdx.x * GRP;
  const int64_t n = G.n, m = G.m;
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    int mode = 1, cur = 0, impl = 0, norepl = 0, shared = 0;
    uint64_t seed = 0;
    uint32_t t0 = 0, t1 = 0;
    for (int g = 0; g < GRP; ++g) {
      const int s = g0 + g;
      if (s >= G.nslots || slots[s].state != 1) continue;
      const Slot *sl = &slots[s];
      const int c = sl->cur;
      const bool exact = c >= sl->R;
      const uint32_t a0 = exact ? 0u : (c ? (uint32_t)sl->T[c - 1] : 0u);
      const uint32_t a1 = exact ? 0u : (uint32_t)sl->T[c];
      if (run == 0) {
        cur = c;
        seed = sl->seed;
        impl = sl->implicit == 1;
        norepl = sl->norepl;
        shared = sl->shared;
        t0 = a0;
        t1 = a1;
        mode = exact ? 2 : 1;
      } else if (c != cur || (exact ? 2 : 1) != mode || (sl->implicit == 1) != (impl != 0) ||
                 (!exact && (sl->seed != seed || sl->norepl != norepl || sl->shared != shared || a0 != t0 ||
                             a1 != t1))) {
        mode = 0;
      }
      run |= 1u << g;
    }
    s_run = run;
    s_norepl = norepl;
    s_shared = shared;
    s_mode = run ? mode : -1;
    s_cur = cur;
    s_impl = impl;
    s_seed = seed;
    s_t0 = t0;
    s_t1 = t1;
  }
  __syncthreads();
  const int mode = s_mode;
  if (mode < 0) return;
  const uint32_t run = s_run;
  // (the exact round on the matrix cores is squared l2 only)
  if (mode == 0 || (mode == 2 && (m > 65536 || MET == KNN_METRIC_L1))) {
    for (int g = 0; g < GRP; ++g)
      if (run & (1u << g))
        sample_slot_chunk<KNN_U8, MET, true, GBT>(&slots[g0 + g], g0 + g, (int64_t)blockIdx.y, X, B, G, smem);
    return;
  }
  const int64_t base = (int64_t)blockIdx.y * G.ch_sample;
  if (base >= n) return;
  const int64_t end = min(n, base + (int64_t)G.ch_sample);
  const int cur = s_cur;
  const int impl = s_impl;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  if (mode == 1) {
    // queries transposed into LDS: qT[j * GRP + g]
    for (int g = 0; g < GRP; ++g) {
      const uint8_t *qg = (run & (1u << g)) ? reinterpret_cast<const uint8_t *>(slots[g0 + g].q) : nullptr;
      for (int64_t j = threadIdx.x; j < m; j += GBT) smem[j * GRP + g] = qg ? qg[j] : 0;
    }
    __syncthreads();
    const uint32_t blk0 = s_t0 >> 2, blk1 = s_t1 >> 2;
    const uint64_t seed = s_seed;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t mm = (uint32_t)m;
    // the grouped kernel runs only for m < 4096, so a round's total per
    // point (B * 255^2) fits in 32 bits
    uint64_t my_pairs = 0, my_pts = 0;
    if (G.stage > 0) {
      // long rounds: tiles of G.stage point rows are copied into LDS with
      // coalesced 16-byte loads and the draws gather from there, so the
      // gathers no longer cost one cache line each in the vector memory
      // path; GBT / G.stage lanes serve one point
      const int TP = G.stage, lpp = GBT / TP;
      const int pt = threadIdx.x / lpp, sub = threadIdx.x % lpp;
      uint8_t *xt = smem + (size_t)GRP * mp;
      for (int64_t tile = base; tile < end; tile += TP) {
        const int rows = (int)min((int64_t)TP, end - tile);
        const uint8_t *src = X + tile * m;
        const int64_t bytes = (int64_t)rows * m;
        if ((m & 15) == 0) {
          for (int64_t v = threadIdx.x; v < bytes / 16; v += GBT)
            reinterpret_cast<uint4 *>(xt)[v] = reinterpret_cast<const uint4 *>(src)[v];
        } else {
          for (int64_t v = threadIdx.x; v < bytes; v += GBT) xt[v] = src[v];
        }
        __syncthreads();
        if (pt < rows) {
          const int32_t i = (int32_t)(tile + pt);
          const uint32_t act = group_active(B, g0, n, i, run, impl);
          if (act) {  // uniform within the lanes of this point
            uint32_t acc[GRP];
            point_sums<MET>(xt + (size_t)pt * m, smem, (uint32_t)i, blk0 + sub, (uint32_t)lpp, blk1, k0, k1, mm, s_norepl,
                       s_shared, acc);
            reduce_store_lpp(lpp, acc, lane, act, g0, n, i, cur, B);
            if (sub == 0) {
              my_pts += 1;
              my_pairs += (uint64_t)__popc(act);
            }
          }
        }
        __syncthreads();
      }
    } else {
      int lpp = G.lpp;
      if (lpp <= 0) {  // about sixteen blocks of draws per lane amortise the per-point work
        const uint32_t nb = blk1 - blk0;
        lpp = 1;
        while (lpp < kWave && (uint32_t)(32 * lpp) <= nb) lpp <<= 1;
      }
      const int sub = threadIdx.x % lpp;
      for (int64_t p = base + threadIdx.x / lpp; p < end; p += GBT / lpp) {
        const int32_t i = (int32_t)p;
        const uint32_t act = group_active(B, g0, n, i, run, impl);
        if (act == 0) continue;  // uniform within the lanes of this point
        uint32_t acc[GRP];
        point_sums<MET>(X + (int64_t)i * m, smem, (uint32_t)i, blk0 + sub, (uint32_t)lpp, blk1, k0, k1, mm, s_norepl,
                   s_shared, acc);
        reduce_store_lpp(lpp, acc, lane, act, g0, n, i, cur, B);
        if (sub == 0) {
          my_pts += 1;
          my_pairs += (uint64_t)__popc(act);
        }
      }
    }
    if (G.prof) {  // whole waves reach this point
      const uint64_t B_r = (uint64_t)(s_t1 - s_t0);
      wave_count_add(&prof_copy(G.prof)[0], my_pairs * (B_r + 21));
      wave_count_add(&prof_copy(G.prof)[1], my_pairs * B_r);
      wave_count_add(&prof_copy(G.prof)[3], my_pts * B_r);
    }
    return;
  }
  // mode 2: exact round on the matrix cores.  Shifted int8 queries,
  // row-major [GRP][mp] in LDS (zero rows for idle slots, zero padding).
  int8_t *Qs = reinterpret_cast<int8_t *>(smem);
  int64_t *qn_s = reinterpret_cast<int64_t *>(smem + (size_t)GRP * mp);
  for (int g = 0; g < GRP; ++g) {
    const uint8_t *qg = (run & (1u << g)) ? reinterpret_cast<const uint8_t *>(slots[g0 + g].q) : nullptr;
    int64_t part = 0;
    for (int64_t j = threadIdx.x; j < mp; j += GBT) {
      const int v = (qg && j < m) ? (int)qg[j] - 128 : 0;
      Qs[(int64_t)g * mp + j] = (int8_t)v;
      part += v * v;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) part += shfl_xor_i64(part, o);
    if (lane == 0) s_qn[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int w = 0; w < GBT / kWave; ++w) t += s_qn[w];
      qn_s[g] = t;
    }
    __syncthreads();
  }
  uint64_t my_pairs = 0;
  const int64_t ntile = (end - base + 15) / 16;
  for (int64_t t = wave; t < ntile; t += GBT / kWave) {
    const int64_t p0 = base + 16 * t;
    const int64_t prow = p0 + (lane & 15);
    const bool pin = prow < end;
    v4i_t acc = v4i_t{0, 0, 0, 0};
    const int8_t *qrow = Qs + (int64_t)(lane & 15) * mp + 16 * (lane >> 4);
    const int8_t *xrow = X8 + (pin ? prow : 0) * mp + 16 * (lane >> 4);
    int64_t k0 = 0;
    for (; k0 + 256 <= mp; k0 += 256) {  // four k-steps per batch of loads
      v4i_t b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        b[u] = pin ? *reinterpret_cast<const v4i_t *>(xrow + k0 + 64 * u) : v4i_t{0, 0, 0, 0};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(*reinterpret_cast<const v4i_t *>(qrow + k0 + 64 * u), b[u],
                                                    acc, 0, 0, 0);
    }
    for (; k0 < mp; k0 += 64) {
      const v4i_t a = *reinterpret_cast<const v4i_t *>(qrow + k0);
      const v4i_t b = pin ? *reinterpret_cast<const v4i_t *>(xrow + k0) : v4i_t{0, 0, 0, 0};
      acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc, 0, 0, 0);
    }
    // lane holds D[g = 4 (lane / 16) + v][point p0 + lane % 16]
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int g = 4 * (lane >> 4) + v;
      if (!pin || !(run & (1u << g))) continue;
      const int64_t off = (int64_t)(g0 + g) * n + prow;
      if (!impl && B.fl[off] != 0) continue;  // not an undecided sampled point of slot g
      B.S[off] = qn_s[g] + (int64_t)xn[prow] - 2 * (int64_t)acc[v];
      if (cur == 0) {
        B.fl[off] = FL_EXACT;
        B.ri[off] = 0;
      } else {
        B.fl[off] = FL_EXACT;
      }
      my_pairs += 1;
    }
  }
  if (G.prof) {  // whole waves reach this point
    wave_count_add(&prof_copy(G.prof)[0], my_pairs * (uint64_t)(m + 14));
    wave_count_add(&prof_copy(G.prof)[2], my_pairs * (uint64_t)m);
  }
}

// ---------------------------------------------------------------- query-lane sample (u8)

// In a sampled round shared by every running slot (one seed, one round:
// the draws of a point are then the same for all of them), one wave serves
// one point for up to 1024 slots, sixteen per lane.  The lanes draw 64
// blocks of four coordinates in parallel (one Philox call each) and the
// gathered x_ij; then, block by block, the coordinates are read back as
// wave-uniform values and every lane loads the sixteen query bytes of its
// slots at each coordinate from the transposed query matrix QT[j][slot]
// (one coalesced 16-byte load per lane; the matrix stays in L2).  Per lane
// the sums use the same x.x - 2 x.q + q.q dot4 form as the grouped kernel
// (for the l1 distance one v_sad_u8 per query and four draws).
constexpr int QL_BT = 256;
constexpr int QL_NW = QL_BT / kWave;
constexpr int QL_SLOTS = 16 * kWave;  // slots served by one wave
constexpr uint32_t QL_NONE = 0xFFFFFFFFu;  // D entry of a pair not sampled this round
constexpr int FT = 64;                     // tile edge of the point-major / slot-major transposes

// A[i][s] = fl[s][i] for the slots running round cur, 1 for the others (a
// nonzero byte means "not sampled"): the point-major copy of the flags that
// the query-lane kernel reads with one 16-byte load per lane.
__global__ __launch_bounds__(NT) void k_flags_ql(const Slot *__restrict__ slots, uint8_t *__restrict__ A, int32_t nqp,
                                                 Bufs B, Geometry G, int32_t cur) {
  __shared__ uint8_t t[FT][FT + 4];
  const int64_t n = G.n;
  const int ns = G.nslots;
  const int64_t i0 = (int64_t)blockIdx.x * FT;
  const int s0 = (int)blockIdx.y * FT;
  const int c = threadIdx.x % FT, r0 = threadIdx.x / FT;
  for (int r = r0; r < FT; r += NT / FT) {  // row r: slot s0 + r, column c: point i0 + c
    const int sl = s0 + r;
    const int64_t i = i0 + c;
    uint8_t v = 1;
    if (sl < ns && i < n && slots[sl].state == 1 && slots[sl].cur == cur) v = B.fl[(int64_t)sl * n + i];
    t[r][c] = v;
  }
  __syncthreads();
  for (int r = r0; r < FT; r += NT / FT) {  // row r: point i0 + r, column c: slot s0 + c
    const int64_t i = i0 + r;
    const int sl = s0 + c;
    if (i < n && sl < nqp) A[i * nqp + sl] = t[c][r];
  }
}

// S[s][i] += D[i][s] (S = D in round 0, with flags cleared), round index
// cur, for the sampled pairs (D != QL_NONE): 64 x 64 tiles transposed through
// LDS so that both the point-major reads and the slot-major writes are
// coalesced.
__global__ __launch_bounds__(NT) void k_fold_ql(const Slot *__restrict__ slots, const uint32_t *__restrict__ D,
                                                int32_t nqp, Bufs B, Geometry G, int32_t cur) {
  __shared__ uint32_t t[FT][FT + 1];
  const int64_t n = G.n;
  const int ns = G.nslots;
  const int64_t i0 = (int64_t)blockIdx.x * FT;
  const int s0 = (int)blockIdx.y * FT;
  const int c = threadIdx.x % FT, r0 = threadIdx.x / FT;
  for (int r = r0; r < FT; r += NT / FT) {
    const int64_t i = i0 + r;
    const int sl = s0 + c;
    t[r][c] = (i < n && sl < nqp) ? D[i * nqp + sl] : QL_NONE;
  }
  __syncthreads();
  for (int r = r0; r < FT; r += NT / FT) {
    const int sl = s0 + r;
    const int64_t i = i0 + c;
    if (sl >= ns || i >= n) continue;
    if (slots[sl].state != 1 || slots[sl].cur != cur) continue;  // D holds nothing of this round for it
    const uint32_t v = t[c][r];
    if (v == QL_NONE) continue;
    const int64_t off = (int64_t)sl * n + i;
    if (cur == 0) {
      B.S[off] = (int64_t)v;
      B.fl[off] = 0;
    } else {
      B.S[off] += (int64_t)v;
    }
    B.ri[off] = (uint8_t)cur;
  }
}

// QT[j * nqp + s] = q_s[j] for the running slots s < ns, 0 elsewhere.
__global__ __launch_bounds__(NT) void k_build_qt(const Slot *__restrict__ slots, int32_t ns, int64_t m, int32_t nqp,
                                                 uint8_t *__restrict__ QT) {
  const int64_t total = m * (int64_t)nqp;
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
    const int64_t j = idx / nqp;
    const int s = (int)(idx - j * nqp);
    uint8_t v = 0;
    if (s < ns && slots[s].state == 1) v = reinterpret_cast<const uint8_t *>(slots[s].q)[j];
    QT[idx] = v;
  }
}

// ------------------------------------------- one sequence for all points

// Boundary b of the gathered copies: T'_0 = 0, T'_b = T[b - 1] for b <= R,
// T'_{R+1} = m (sampling without replacement: the exact round's remaining
// coordinates).
__device__ __forceinline__ int64_t seq_boundary(const Sched *sc, int b, int64_t m) {
  return b == 0 ? 0 : (b <= sc->R ? (int64_t)sc->T[b - 1] : m);
}

// Coordinate of sample t of the sequence every point shares (counter words
// (0, 2), or the permutation keyed by (0, 3)), for t < tlen; ~0u for t in
// [tlen, kp).
__global__ __launch_bounds__(NT) void k_seq_coords(uint64_t seed, int32_t norepl, int64_t m, int32_t tlen,
                                                   int64_t kp, uint32_t *__restrict__ js) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32), mm = (uint32_t)m;
  const int ph = perm_half_bits(mm);
  const PermKey pk = norepl ? perm_key(0u, draw_c3(true, true), k0, k1) : PermKey{{0u, 0u, 0u, 0u}};
  for (int64_t b = (int64_t)blockIdx.x * NT + threadIdx.x; 4 * b < kp; b += (int64_t)gridDim.x * NT) {
    uint32_t j4[4] = {~0u, ~0u, ~0u, ~0u};
    if (4 * b + 4 <= tlen || (!norepl && 4 * b < tlen)) {
      draw_block((uint32_t)b, 0u, draw_c3(true, false), k0, k1, mm, norepl != 0, ph, pk, j4);
    } else if (4 * b < tlen) {
      // the last, partial block of a permutation: only positions below
      // tlen = m (the cycle walk from a position >= m need not return below m)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (4 * b + e < tlen) j4[e] = perm_coord((uint32_t)(4 * b + e), mm, ph, pk);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) js[4 * b + e] = 4 * b + e < tlen ? j4[e] : ~0u;
  }
}

// Rows at the sequence's coordinates, out[r][t] = row_r[js[t]] (as x - 128
// for squared l2, raw bytes for l1; zero where js[t] is none): the points
// (rows = n), or the running slots' queries (QUERIES, rows = nqp; idle
// slots give zero rows).  One row per block at a time: with STAGE the row
// is read into LDS by the whole block (a point row as the aligned 16-byte
// words that cover it, at any m; a query row with 16-, 4- or 1-byte loads
// as its alignment allows) and the coordinates are kept in LDS as 16-bit values
// (m < 65536; 0xFFFF: none); each thread then gathers sixteen bytes per
// step.  Without STAGE the bytes come from the row in global memory.  BT
// threads per block: 1024 for staged rows whose LDS leaves room for fewer
// than four blocks per CU, so that enough loads are in flight, else 256.  Only the columns
// [c0, c1) (multiples of 16) are written, and only their coordinates are
// held in LDS; with `need` set and *need == 0 the launch does nothing.
template <int MET, bool QUERIES, bool STAGE, int BT = NT>
__global__ __launch_bounds__(BT) void k_seq_gather(const uint8_t *__restrict__ X, const Slot *__restrict__ slots,
                                                   int32_t ns, int64_t rows, int64_t m,
                                                   const uint32_t *__restrict__ js, int64_t kp,
                                                   int8_t *__restrict__ out, int64_t c0, int64_t c1,
                                                   const int32_t *__restrict__ need) {
  if (need && *need == 0) return;
  extern __shared__ __align__(16) uint8_t srow[];
  const int64_t mr = (m + 15) / 16 * 16;
  uint16_t *jl = reinterpret_cast<uint16_t *>(srow + (STAGE ? mr + 16 : 0));
  if constexpr (STAGE) {
    for (int64_t t = c0 + threadIdx.x; t < c1; t += BT) jl[t - c0] = js[t] == ~0u ? (uint16_t)0xFFFFu : (uint16_t)js[t];
    __syncthreads();
  }
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const uint8_t *row = nullptr;  // (block-uniform)
    if constexpr (QUERIES) {
      if (r < ns && slots[r].state == 1) row = reinterpret_cast<const uint8_t *>(slots[r].q);
    } else {
      row = X + r * m;
    }
    int64_t shift = 0;  // the row's offset in its staged copy (block-uniform)
    if constexpr (STAGE) {
      if (!QUERIES) {
        // the aligned 16-byte words that cover the row, read whole where they
        // lie inside the matrix (at either end of an unaligned row they hold
        // bytes of the next or previous row, which nothing reads); bytes of
        // a word that reaches past the matrix are read one by one
        shift = (int64_t)((uintptr_t)row & 15);
        const uint8_t *base = row - shift, *end = X + rows * m;
        const int64_t nw = (shift + m + 15) / 16;
        for (int64_t w = threadIdx.x; w < nw; w += BT) {
          const uint8_t *p = base + 16 * w;
          if (p >= X && p + 16 <= end) {
            reinterpret_cast<uint4 *>(srow)[w] = *reinterpret_cast<const uint4 *>(p);
          } else {
            for (int e = 0; e < 16; ++e)
              if (p + e >= row && p + e < row + m) srow[16 * w + e] = p[e];
          }
        }
      } else if (row) {
        const uintptr_t al = (uintptr_t)row;
        if ((m & 15) == 0 && (al & 15) == 0) {
          for (int64_t w = threadIdx.x; w < m / 16; w += BT)
            reinterpret_cast<uint4 *>(srow)[w] = reinterpret_cast<const uint4 *>(row)[w];
        } else if ((m & 3) == 0 && (al & 3) == 0) {
          for (int64_t w = threadIdx.x; w < m / 4; w += BT)
            reinterpret_cast<uint32_t *>(srow)[w] = reinterpret_cast<const uint32_t *>(row)[w];
        } else {
          for (int64_t j = threadIdx.x; j < m; j += BT) srow[j] = row[j];
        }
      }
      __syncthreads();
    }
    const uint8_t *from = STAGE ? srow + shift : row;
    for (int64_t t0 = c0 + 16 * (int64_t)threadIdx.x; t0 < c1; t0 += 16 * BT) {
      uint32_t jj[16];
      if constexpr (STAGE) {
        const uint4 *jp = reinterpret_cast<const uint4 *>(jl + (t0 - c0));
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const uint4 j = jp[d];
          const uint32_t hw[4] = {j.x, j.y, j.z, j.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t lo = hw[e] & 0xFFFFu, hi = hw[e] >> 16;
            jj[8 * d + 2 * e] = lo == 0xFFFFu ? ~0u : lo;
            jj[8 * d + 2 * e + 1] = hi == 0xFFFFu ? ~0u : hi;
          }
        }
      } else {
        const uint4 *jp = reinterpret_cast<const uint4 *>(js + t0);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const uint4 j = jp[d];
          jj[4 * d] = j.x;
          jj[4 * d + 1] = j.y;
          jj[4 * d + 2] = j.z;
          jj[4 * d + 3] = j.w;
        }
      }
      uint32_t w[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        uint32_t word = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t j = jj[4 * d + e];
          uint32_t v = 0;
          if (row && j != ~0u) v = MET == KNN_METRIC_L2 ? (uint32_t)(from[j] ^ 0x80u) : (uint32_t)from[j];
          word |= v << (8 * e);
        }
        w[d] = word;
      }
      *reinterpret_cast<uint4 *>(out + r * kp + t0) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if constexpr (STAGE) __syncthreads();  // the row buffer is refilled next
  }
}

// Sampled rounds of the sparse slots of a point-major batch whose queries
// share one coordinate sequence: the samples [t0, t1) of pair (s, i) are
// columns t0..t1-1 of the gathered rows XS[i] and QS[s], so the round sum is
// a contiguous sum over those bytes (no draws).  Lanes per point: enough
// for one 4-byte word per lane and step, up to a whole wave.  The sums go
// to the slot-major running sums, like k_sample's.
constexpr int SEQ_SP = 64;  // list entries per block of k_sample_seq_sparse

template <int MET>
__global__ __launch_bounds__(NT) void k_sample_seq_sparse(const Slot *__restrict__ slots, SeqBufs q, Bufs B,
                                                          Geometry G) {
  const int s = blockIdx.x;
  const Slot *sl = &slots[s];
  if (sl->state != 1 || sl->implicit != 0) return;  // dense slots run the tiled round
  const int cur = sl->cur;
  if (cur >= sl->R) return;  // the exact round takes the per-slot exact pass
  const int64_t n = G.n;
  const SlotArrays a = slot_arrays(B, n, s, sl->par);
  const int64_t nlist = sl->n_act;
  const int64_t w0 = (cur ? (int64_t)sl->T[cur - 1] : 0) / 4, w1 = (int64_t)sl->T[cur] / 4;
  const int64_t words = w1 - w0;
  const int lpp = words <= 16 ? 16 : (words <= 32 ? 32 : kWave);
  const int sub = threadIdx.x % lpp;
  const uint32_t *qrow = reinterpret_cast<const uint32_t *>(q.qs + (int64_t)s * q.kp);
  uint64_t my_pts = 0;
  for (int64_t c = blockIdx.y; c * SEQ_SP < nlist; c += gridDim.y) {
    const int64_t base = c * SEQ_SP, end = min(nlist, base + (int64_t)SEQ_SP);
    for (int64_t p = base + threadIdx.x / lpp; p < end; p += NT / lpp) {
      const int32_t i = a.act[p];
      const uint32_t *xrow = reinterpret_cast<const uint32_t *>(q.xs + (int64_t)i * q.kp);
      uint32_t acc = 0;  // below 2^32: at most m < 65536 samples of at most 255^2
      for (int64_t w = w0 + sub; w < w1; w += lpp) {
        if constexpr (MET == KNN_METRIC_L1) {
          acc = __builtin_amdgcn_sad_u8(xrow[w], qrow[w], acc);
        } else {
          const uint32_t xu = xrow[w] ^ 0x80808080u, qu = qrow[w] ^ 0x80808080u;  // back to unsigned bytes
          acc += __builtin_amdgcn_udot4(xu, xu, 0u, false) + __builtin_amdgcn_udot4(qu, qu, 0u, false) -
                 2u * __builtin_amdgcn_udot4(xu, qu, 0u, false);
        }
      }
      for (int o = lpp / 2; o > 0; o >>= 1) acc += (uint32_t)__shfl_xor((int)acc, o);
      if (sub == 0) {
        a.S[i] += (int64_t)acc;
        a.ri[i] = (uint8_t)cur;
        ++my_pts;
      }
    }
  }
  if (G.prof && my_pts) atomicAdd(&prof_copy(G.prof)[1], my_pts * (uint64_t)(4 * words));
}

// Float rows at the sequence's coordinates, out[r][t] = row_r[js[t]] (zero
// where js[t] is none): the points (rows = n) or the running slots' queries
// (QUERIES, rows = ns).  One row per block at a time, staged in LDS when
// STAGE (m floats).
template <bool QUERIES, bool STAGE>
__global__ __launch_bounds__(NT) void k_seq_gather_f32(const float *__restrict__ X, const Slot *__restrict__ slots,
                                                       int64_t rows, int64_t m, const uint32_t *__restrict__ js,
                                                       int64_t kp, float *__restrict__ out) {
  extern __shared__ __align__(16) float frow[];
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const float *row = nullptr;  // (block-uniform)
    if constexpr (QUERIES) {
      if (slots[r].state == 1) row = reinterpret_cast<const float *>(slots[r].q);
    } else {
      row = X + r * m;
    }
    if constexpr (STAGE) {
      if (row)
        for (int64_t j = threadIdx.x; j < m; j += NT) frow[j] = row[j];
      __syncthreads();
    }
    const float *from = STAGE ? frow : row;
    for (int64_t t = threadIdx.x; t < kp; t += NT) {
      const uint32_t j = js[t];
      out[r * kp + t] = (row && j != ~0u) ? from[j] : 0.0f;
    }
    if constexpr (STAGE) __syncthreads();
  }
}

// Squared norms of gathered rows (x - 128 bytes) over the samples before
// each boundary: out[b * ostride + r] = sum_{t < T'_b} S[r][t]^2 for b < nb.
// The boundary T'_{R+1} = m (sampling without replacement) is the full-row
// norm, copied from `full` (the points' or queries' norms of the naive
// scan) instead of summed.  One wave per row.  When the summed boundaries'
// words fit NRW words per lane (up to 4 KB of a row), a lane loads all of
// its words at once and each boundary's sum is taken from their squares
// in registers; longer ranges take one boundary at a time.
__global__ __launch_bounds__(NT) void k_seq_norms(const int8_t *__restrict__ S, int64_t rows, int64_t kp,
                                                  const Sched *__restrict__ sc, int32_t nb, int64_t m,
                                                  const int32_t *__restrict__ full, int32_t *__restrict__ out,
                                                  int64_t ostride, int32_t b_lo, int32_t b_hi,
                                                  const int32_t *__restrict__ need) {
  // boundaries b_lo <= b < min(b_hi, nb), continuing from boundary b_lo - 1
  if (need && *need == 0) return;
  constexpr int NRW = 16;
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * (NT / kWave);
  // boundaries [bs, bx) are summed; R + 1 (the last), when below be, is copied
  const int bs = std::max(1, (int)b_lo), be = min((int)b_hi, (int)nb), bx = min(be, sc->R + 1);
  // words [wa, wz) of the summed boundaries: T'_{b-1} is a multiple of 4, and
  // bytes past the last sample are zero
  const int64_t wa = bs < bx ? seq_boundary(sc, bs - 1, m) / 4 : 0;
  const int64_t wz = bs < bx ? (seq_boundary(sc, bx - 1, m) + 3) / 4 : 0;
  const bool held = wz - wa <= (int64_t)kWave * NRW;
  if (bs >= bx) {  // nothing to sum: boundary 0 and the full-row boundary at most, one thread per row
    for (int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x; r < rows; r += (int64_t)gridDim.x * NT) {
      if (b_lo <= 1) out[r] = 0;
      if (bs <= bx && bx < be) out[(int64_t)bx * ostride + r] = full[r];
    }
    return;
  }
  for (int64_t r = (int64_t)blockIdx.x * (NT / kWave) + threadIdx.x / kWave; r < rows; r += nw) {
    const uint32_t *row = reinterpret_cast<const uint32_t *>(S + r * kp);
    int32_t run = b_lo > 1 ? out[(int64_t)(b_lo - 1) * ostride + r] : 0;
    if (lane == 0 && b_lo <= 1) out[r] = 0;
    if (held) {
      // the squares of word wa + lane + 64 j (one signed 4-byte dot product
      // each), then each boundary's sum over [wa, T'_b) from them
      int32_t sq[NRW];
#pragma unroll
      for (int j = 0; j < NRW; ++j) {
        const int32_t w = (int32_t)wa + lane + kWave * j;
        const int32_t v = w < (int32_t)wz ? (int32_t)row[w] : 0;
        sq[j] = __builtin_amdgcn_sdot4(v, v, 0, false);
      }
      const int32_t base = run;
      for (int b = bs; b < bx; ++b) {
        const int32_t w1 = (int32_t)((seq_boundary(sc, b, m) + 3) / 4);
        int32_t part = 0;
#pragma unroll
        for (int j = 0; j < NRW; ++j) part += ((int32_t)wa + lane + kWave * j < w1) ? sq[j] : 0;
        for (int o = kWave / 2; o > 0; o >>= 1) part += __shfl_xor(part, o);
        run = base + part;
        if (lane == 0) out[(int64_t)b * ostride + r] = run;
      }
      if (bs <= bx && bx < be && lane == 0) out[(int64_t)bx * ostride + r] = full[r];  // bx = R + 1: all m coordinates
      continue;
    }
    for (int b = bs; b < be; ++b) {
      if (b == sc->R + 1) {  // all m coordinates
        if (lane == 0) out[(int64_t)b * ostride + r] = full[r];
        continue;
      }
      const int64_t w0 = seq_boundary(sc, b - 1, m) / 4, w1 = (seq_boundary(sc, b, m) + 3) / 4;
      int32_t part = 0;
      for (int64_t w = w0 + lane; w < w1; w += kWave) {
        const uint32_t v = row[w];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int32_t x = (int32_t)(int8_t)(v >> (8 * e));
          part += x * x;
        }
      }
      for (int o = kWave / 2; o > 0; o >>= 1) part += __shfl_xor(part, o);
      run += part;
      if (lane == 0) out[(int64_t)b * ostride + r] = run;
    }
  }
}

template <int MET>
__global__ __launch_bounds__(QL_BT) void k_sample_ql_u8(const Slot *__restrict__ slots, const uint8_t *__restrict__ X,
                                                        const uint8_t *__restrict__ QT, int32_t nqp,
                                                        const uint8_t *__restrict__ A, uint32_t *__restrict__ D,
                                                        Bufs B, Geometry G, QlRound R) {
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int64_t n = G.n, m = G.m;
  const int ns = G.nslots;
  const int s0 = (int)blockIdx.y * QL_SLOTS + 16 * lane;
  const bool has_q = s0 < nqp;  // nqp is a multiple of 16; other lanes read column 0 and store nothing
  uint32_t run = 0;
  for (int g = 0; g < GRP; ++g) {
    const int s = s0 + g;
    if (s < ns && slots[s].state == 1 && slots[s].cur == R.cur && (!G.flagsets || slots[s].implicit != 0))
      run |= 1u << g;
  }
  if (__ballot(run != 0) == 0) return;  // no running slot in this wave's range
  const uint32_t blk0 = R.t0 >> 2, blk1 = R.t1 >> 2;
  const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);
  const uint32_t mm = (uint32_t)m;
  const bool norepl = R.norepl != 0, shared = R.shared != 0;
  const int ph = perm_half_bits(mm);
  const uint32_t c3 = draw_c3(shared, false);
  // QT through a buffer descriptor: the row offset j * nqp is a wave-uniform
  // scalar and the lane's column a fixed vector offset, so a load costs no
  // address arithmetic (and reads past the matrix return zeros)
  const __amdgpu_buffer_rsrc_t qrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(QT), 0, (int)(m * nqp), 0x00020000);
  const int qcol = has_q ? s0 : 0;  // this lane's sixteen columns
  uint64_t my_pairs = 0, my_pts = 0;
  // each block walks a contiguous range of points, its waves interleaved, so
  // that the per-slot rows of S, flags and rounds it updates (one 128-byte
  // line holds 16 consecutive points) are written from one L2 in a short time
  const int64_t per_block = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i_end = min(n, ((int64_t)blockIdx.x + 1) * per_block);
  // the next point's "not sampled" bytes are loaded while this point is
  // sampled (prefetching its old sums too measured no faster: the 16 more
  // registers cost a wave per SIMD)
  uint4 a_next = make_uint4(0u, 0u, 0u, 0u);
  const int64_t i_first = (int64_t)blockIdx.x * per_block + wave;
  if (!R.impl && i_first < i_end) a_next = *reinterpret_cast<const uint4 *>(A + i_first * (int64_t)nqp + qcol);
  for (int64_t i = i_first; i < i_end; i += QL_NW) {
    const uint4 a_cur = a_next;
    if (!R.impl && i + QL_NW < i_end)
      a_next = *reinterpret_cast<const uint4 *>(A + (i + QL_NW) * (int64_t)nqp + qcol);
    // undecided sampled pairs: zero bytes of the point-major flag copy
    uint32_t act = run;
    if (!R.impl) {
      const uint4 a = a_cur;
      const uint32_t w[4] = {a.x, a.y, a.z, a.w};
      act = 0;
#pragma unroll
      for (int g = 0; g < GRP; ++g) act |= (((w[g >> 2] >> (8 * (g & 3))) & 255u) == 0 ? 1u : 0u) << g;
      act &= run;
    }
    uint4 *drow = reinterpret_cast<uint4 *>(D + i * (int64_t)nqp + qcol);
    if (__ballot(act != 0) == 0) {  // wave-uniform: nothing to sample at this point
      if (has_q && !G.flagsets) {
        const uint4 none = make_uint4(QL_NONE, QL_NONE, QL_NONE, QL_NONE);
#pragma unroll
        for (int c = 0; c < 4; ++c) drow[c] = none;
      }
      continue;
    }
    const uint8_t *row = X + i * m;
    const uint32_t c2 = draw_c2((uint32_t)i, shared);
    const PermKey pk = norepl ? perm_key(c2, draw_c3(shared, true), k0, k1) : PermKey{{0u, 0u, 0u, 0u}};
    uint32_t qq[GRP], xq[GRP], xx = 0;
#pragma unroll
    for (int g = 0; g < GRP; ++g) qq[g] = xq[g] = 0;
    for (uint32_t bb = blk0; bb < blk1; bb += kWave) {
      // lane l draws block bb + l
      uint32_t jv[4] = {0u, 0u, 0u, 0u}, xv = 0;
      if (bb + lane < blk1) {
        draw_block(bb + lane, c2, c3, k0, k1, mm, norepl, ph, pk, jv);
        xv = (uint32_t)row[jv[0]] | ((uint32_t)row[jv[1]] << 8) | ((uint32_t)row[jv[2]] << 16) |
             ((uint32_t)row[jv[3]] << 24);
      }
      const int nb = (int)min((uint32_t)kWave, blk1 - bb);
      auto fetch = [&](int d, uint4 (&qv)[4]) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t j = (uint32_t)__builtin_amdgcn_readlane((int)jv[e], d);
          const v4u_t w = __builtin_amdgcn_raw_buffer_load_b128(qrs, qcol, (int)(j * (uint32_t)nqp), 0);
          qv[e] = make_uint4(w.x, w.y, w.z, w.w);
        }
      };
      auto consume = [&](int d, const uint4 (&qv)[4]) {
        const uint32_t x4 = (uint32_t)__builtin_amdgcn_readlane((int)xv, d);
        if constexpr (MET == KNN_METRIC_L2) xx = __builtin_amdgcn_udot4(x4, x4, xx, false);
        const uint32_t r[4][4] = {{qv[0].x, qv[1].x, qv[2].x, qv[3].x},
                                  {qv[0].y, qv[1].y, qv[2].y, qv[3].y},
                                  {qv[0].z, qv[1].z, qv[2].z, qv[3].z},
                                  {qv[0].w, qv[1].w, qv[2].w, qv[3].w}};
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t t0 = __builtin_amdgcn_perm(r[w][1], r[w][0], 0x05010400u);
          const uint32_t t1 = __builtin_amdgcn_perm(r[w][1], r[w][0], 0x07030602u);
          const uint32_t t2 = __builtin_amdgcn_perm(r[w][3], r[w][2], 0x05010400u);
          const uint32_t t3 = __builtin_amdgcn_perm(r[w][3], r[w][2], 0x07030602u);
          const uint32_t c[4] = {__builtin_amdgcn_perm(t2, t0, 0x05040100u), __builtin_amdgcn_perm(t2, t0, 0x07060302u),
                                 __builtin_amdgcn_perm(t3, t1, 0x05040100u), __builtin_amdgcn_perm(t3, t1, 0x07060302u)};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if constexpr (MET == KNN_METRIC_L1) {
              xq[4 * w + u] = __builtin_amdgcn_sad_u8(x4, c[u], xq[4 * w + u]);
            } else {
              qq[4 * w + u] = __builtin_amdgcn_udot4(c[u], c[u], qq[4 * w + u], false);
              xq[4 * w + u] = __builtin_amdgcn_udot4(x4, c[u], xq[4 * w + u], false);
            }
          }
        }
      };
      // three register stages: the loads of blocks d + 1 and d + 2 are in
      // flight while d is summed (issued unconditionally, the last block
      // again at the end, so that the wait before each sum covers only the
      // oldest stage)
      uint4 qa[4], qb[4], qc[4];
      fetch(0, qa);
      fetch(min(1, nb - 1), qb);
      int d = 0;
      for (;;) {
        fetch(min(d + 2, nb - 1), qc);
        consume(d, qa);
        if (++d >= nb) break;
        fetch(min(d + 2, nb - 1), qa);
        consume(d, qb);
        if (++d >= nb) break;
        fetch(min(d + 2, nb - 1), qb);
        consume(d, qc);
        if (++d >= nb) break;
      }
    }
    // totals of this round per slot (below 2^32 - 1 because m < 66052), in
    // the point-major buffer D (one coalesced 64-byte store per lane): as
    // this round's totals, which the fold kernel adds to the slot-major
    // running sums; or, in batches that keep their sums point-major
    // (G.flagsets), added to D itself, which then holds the running sums
    if (has_q) {
      uint32_t t[GRP], old[GRP];
      if (G.flagsets && !R.impl) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint4 o = drow[c];
          old[4 * c] = o.x;
          old[4 * c + 1] = o.y;
          old[4 * c + 2] = o.z;
          old[4 * c + 3] = o.w;
        }
      } else {
#pragma unroll
        for (int g = 0; g < GRP; ++g) old[g] = G.flagsets ? 0u : QL_NONE;
      }
#pragma unroll
      for (int g = 0; g < GRP; ++g) {
        const uint32_t tot = MET == KNN_METRIC_L1 ? xq[g] : xx + qq[g] - 2u * xq[g];
        t[g] = (act & (1u << g)) ? (G.flagsets ? old[g] + tot : tot) : old[g];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) drow[c] = make_uint4(t[4 * c], t[4 * c + 1], t[4 * c + 2], t[4 * c + 3]);
    }
    my_pairs += (uint64_t)__popc(act);
    if (lane == 0) my_pts += 1;
  }
  if (G.prof) {  // whole waves reach this point (a wave with nothing to do left together)
    const uint64_t B_r = (uint64_t)(R.t1 - R.t0);
    wave_count_add(&prof_copy(G.prof)[0], my_pairs * (B_r + 21));
    wave_count_add(&prof_copy(G.prof)[1], my_pairs * B_r);
    wave_count_add(&prof_copy(G.prof)[3], my_pts * B_r);
  }
}

// ---------------------------------------------------------------- selection

// Writes the K smallest keys of the block (with multiplicity) to out[0..K);
// UINT64_MAX marks padding.  Fast path (K <= 64): the K-th smallest of a
// wave's per-lane minima bounds the block's K-th smallest key from above,
// and so does the least such bound over the waves (tau).  Only the real keys
// at or below tau (usually a few times K) are then ordered, by one wave when
// they fit in it.  The radix selections are the fallbacks.
constexpr int CAND_CAP = 2048;

template <int E>
__device__ void emit_smallest(const uint64_t (&key)[E], int K, uint64_t *out, SelScratch &ss, int &cnt,
                              uint64_t *cand, uint64_t *wtau) {
  constexpr uint64_t PAD = ~0ull;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  int less;
  uint64_t v;
  bool done = false;
  if (K <= kWave) {
    uint64_t mn = key[0];
#pragma unroll
    for (int e = 1; e < E; ++e) mn = key[e] < mn ? key[e] : mn;
    const uint64_t tw = wave_bcast_u64(wave_sort_u64(mn), K - 1);
    if (lane == 0) wtau[wave] = tw;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    uint64_t tau = wtau[0];
#pragma unroll
    for (int w = 1; w < NT / kWave; ++w) tau = wtau[w] < tau ? wtau[w] : tau;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (key[e] <= tau && key[e] != PAD) {
        const int pos = atomicAdd(&cnt, 1);
        if (pos < CAND_CAP) cand[pos] = key[e];
      }
    }
    __syncthreads();
    const int c = cnt;
    __syncthreads();
    if (c <= kWave) {
      if (wave == 0) {
        const uint64_t sv = wave_sort_u64(lane < c ? cand[lane] : PAD);
        if (lane < K) out[lane] = sv;  // PAD beyond the real keys
      }
      __syncthreads();
      return;
    }
    if (c <= CAND_CAP) {
      v = block_kth_gen<NT>(c, [&](int64_t p) { return cand[p]; }, K, ss, &less);
      if (threadIdx.x == 0) cnt = 0;
      __syncthreads();
      for (int p = threadIdx.x; p < c; p += NT)
        if (cand[p] < v) out[atomicAdd(&cnt, 1)] = cand[p];
      done = true;
    }
  }
  if (!done) {
    v = block_kth_regs<NT, E>(key, K, ss, &less);
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (key[e] < v) out[atomicAdd(&cnt, 1)] = key[e];
  }
  for (int j = less + (int)threadIdx.x; j < K; j += NT) out[j] = v;
  __syncthreads();
}

constexpr int SEL_E = 16;
constexpr int SEL_CH = NT * SEL_E;

// Per chunk of P: the k smallest upper bounds and the k+1 smallest lower
// bounds (values).  U, L1, L2 of the whole set are order statistics of the
// union of these lists.
__device__ void select_partial_chunk(const Slot *sl, int s, int64_t chunk, int64_t nP, const Bufs &B,
                                     const Geometry &G) {
  const int64_t n = G.n, m = G.m;
  const int64_t base = chunk * SEL_CH;
  const SlotArrays a = slot_arrays(B, n, s, sl->par);
  __shared__ SelScratch ss;
  __shared__ int cnt;
  __shared__ uint64_t cand[CAND_CAP];
  __shared__ uint64_t wtau[NT / kWave];
  uint64_t ku[SEL_E], kl[SEL_E];
#pragma unroll
  for (int e = 0; e < SEL_E; ++e) {
    const int64_t p = base + (int64_t)e * NT + threadIdx.x;
    if (p < nP) {
      const int32_t i = elem_P(sl, a, p);
      double d, al;
      point_bounds(sl, m, a.S[i], a.fl[i], a.ri[i], d, al);
      ku[e] = dkey(d + al);
      kl[e] = dkey(d - al);
    } else {
      ku[e] = ~0ull;
      kl[e] = ~0ull;
    }
  }
  const int k = sl->k;
  uint64_t *out = B.part + (int64_t)s * B.part_stride + chunk * (2 * k + 1);
  emit_smallest<SEL_E>(ku, k, out, ss, cnt, cand, wtau);
  emit_smallest<SEL_E>(kl, k + 1, out + k, ss, cnt, cand, wtau);
}

// One partial list per SEL_CH elements of P: chunks blockIdx.x,
// blockIdx.x + gridDim.x, ... of the slot's P.
__global__ __launch_bounds__(NT) void k_select_partial(Slot *__restrict__ slots, Bufs B, Geometry G) {
  const int s = blockIdx.y;
  const Slot *sl = &slots[s];
  if (sl->state != 1) return;
  if (G.flagsets && sl->implicit != 0) return;  // a dense slot of a point-major batch
  const int64_t nP = size_P(sl, G.n);
  for (int64_t c = blockIdx.x; c * SEL_CH < nP; c += gridDim.x) {
    select_partial_chunk(sl, s, c, nP, B, G);
    __syncthreads();  // the next chunk reuses the block's LDS
  }
}

// Tiles of the selection over point-major sums (k_select_pm): FS_SL slots x
// FS_PT points, one wave per slot (FS_NT threads), sixteen points per lane;
// the kept set P is exactly the points without a discard flag.  Needs
// k + 1 <= 64 (the wave selection below).  A tile reads FS_SL * 4 bytes of
// each point's line of D: the staging is bound by the number of lines a
// block touches (per launch over 100,000 points x 1,024 slots, the staging
// alone: 4 slots 173 us, 8 slots 126 us, 16 slots 117 us), the
// selections by the vector ALU (111 us without the loads), and the two
// overlap only across blocks resident on a CU together.  Per launch with
// both: 4 slots 197 us, 8 slots 174 us, 16 slots 204 us (two 1024-thread
// blocks per CU, which leaves the loads of one block little to overlap).
constexpr int FS_SL = 8, FS_PT = 1024;
constexpr int FS_NT = FS_SL * kWave;
constexpr int FS_E = FS_PT / kWave;

// The K (<= 64) smallest of the wave's E keys per lane (PAD = none), written
// ascending to out[0..K) (PAD beyond the real keys).  The K-th smallest of
// the lanes' minima bounds the K-th smallest key; the keys at or below it are
// ordered by one wave sort when they fit, else by sorting each key column and
// merging the sorted columns (keeping the 64 smallest).
template <int E>
__device__ void wave_smallest(const uint64_t (&key)[E], int K, uint64_t *out, uint64_t *cbuf) {
  constexpr uint64_t PAD = ~0ull;
  const int lane = lane_id();
  uint64_t mn = key[0];
#pragma unroll
  for (int e = 1; e < E; ++e) mn = key[e] < mn ? key[e] : mn;
  const uint64_t tau = wave_bcast_u64(wave_sort_u64(mn), K - 1);
  int cnt = 0;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool c = key[e] <= tau && key[e] != PAD;
    const uint64_t mk = __ballot(c);
    const int pos = cnt + __popcll(mk & lt);
    if (c && pos < kWave) cbuf[pos] = key[e];
    cnt += __popcll(mk);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint64_t best;
  if (cnt <= kWave) {
    best = wave_sort_u64(lane < cnt ? cbuf[lane] : PAD);
  } else {
    best = wave_sort_u64(key[0]);
#pragma unroll
    for (int e = 1; e < E; ++e) {
      const uint64_t c = wave_sort_u64(key[e]);
      const uint64_t r = wave_bcast_rev_u64(c);  // descending
      uint64_t v = best < r ? best : r;          // bitonic: the 64 smallest of both
#pragma unroll
      for (int j = kWave / 2; j > 0; j >>= 1) {
        const uint64_t o = lane_xor_u64(v, j);
        v = ((lane & j) == 0) ? (o < v ? o : v) : (o > v ? o : v);
      }
      best = v;
    }
  }
  if (lane < K) out[lane] = best;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();  // cbuf is reused by the next call
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The K (<= 64) smallest of N keys get(p), p in [0, N) (PAD = ~0 is no
// key), ascending across the lanes (PAD past the real keys); the method of
// wave_smallest with the keys read twice instead of held in registers.
template <typename Get>
__device__ uint64_t wave_smallest_gen(int64_t N, Get get, int K, uint64_t *cbuf) {
  constexpr uint64_t PAD = ~0ull;
  const int lane = lane_id();
  uint64_t mn = PAD;
  for (int64_t p = lane; p < N; p += kWave) {
    const uint64_t v = get(p);
    mn = v < mn ? v : mn;
  }
  const uint64_t tau = wave_bcast_u64(wave_sort_u64(mn), K - 1);
  int cnt = 0;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  for (int64_t p0 = 0; p0 < N; p0 += kWave) {  // wave-uniform trip count
    const int64_t p = p0 + lane;
    const uint64_t v = p < N ? get(p) : PAD;
    const bool c = v <= tau && v != PAD;
    const uint64_t mk = __ballot(c);
    const int pos = cnt + __popcll(mk & lt);
    if (c && pos < kWave) cbuf[pos] = v;
    cnt += __popcll(mk);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint64_t best = PAD;
  if (cnt <= kWave) {
    best = wave_sort_u64(lane < cnt ? cbuf[lane] : PAD);
  } else {
    for (int64_t p0 = 0; p0 < N; p0 += kWave) {
      const int64_t p = p0 + lane;
      const uint64_t c = wave_sort_u64(p < N ? get(p) : PAD);
      const uint64_t r = wave_bcast_rev_u64(c);  // descending
      uint64_t v = best < r ? best : r;          // bitonic: the 64 smallest of both
#pragma unroll
      for (int j = kWave / 2; j > 0; j >>= 1) {
        const uint64_t o = lane_xor_u64(v, j);
        v = ((lane & j) == 0) ? (o < v ? o : v) : (o > v ? o : v);
      }
      best = v;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();  // cbuf is reused by the next call
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return best;
}

// ---- selections of up to 128 keys: a 128-key list is two registers per
// lane, sorted ascending with lane l holding ranks l (lo) and 64 + l (hi).
__device__ __forceinline__ uint32_t lx(uint32_t v, int j) { return lane_xor_u32(v, j); }
__device__ __forceinline__ uint64_t lx(uint64_t v, int j) { return lane_xor_u64(v, j); }
__device__ __forceinline__ uint32_t wsort(uint32_t v) { return wave_sort_u32(v); }
__device__ __forceinline__ uint64_t wsort(uint64_t v) { return wave_sort_u64(v); }
__device__ __forceinline__ uint32_t wrev(uint32_t v) { return lane_rev_u32(v); }
__device__ __forceinline__ uint64_t wrev(uint64_t v) { return wave_bcast_rev_u64(v); }
__device__ __forceinline__ uint32_t wbcast(uint32_t v, int src) { return (uint32_t)__builtin_amdgcn_readlane((int)v, src); }
__device__ __forceinline__ uint64_t wbcast(uint64_t v, int src) { return wave_bcast_u64(v, src); }

// A sequence bitonic across the lanes, sorted ascending.
template <typename T>
__device__ __forceinline__ T bitonic_clean(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int j = kWave / 2; j > 0; j >>= 1) {
    const T o = lx(v, j);
    v = ((lane & j) == 0) ? (o < v ? o : v) : (o > v ? o : v);
  }
  return v;
}

// Two sorted 64-key columns a, b -> the sorted 128-key list (lo, hi).
template <typename T>
__device__ __forceinline__ void merge64x2(T a, T b, T &lo, T &hi) {
  const T rb = wrev(b);  // a ascending, rb descending: min / max are the two bitonic halves
  lo = bitonic_clean(a < rb ? a : rb);
  hi = bitonic_clean(a < rb ? rb : a);
}

// The 128 smallest of a sorted 128-key list (lo, hi) and a sorted 64-key
// column c, sorted (c is taken as padded to 128 with keys above all).
template <typename T>
__device__ __forceinline__ void merge128_col(T &lo, T &hi, T c) {
  const T rc = wrev(c);
  const T h2 = hi < rc ? hi : rc;  // (lo, h2): the 128 smallest, bitonic
  const T a = lo < h2 ? lo : h2, b = lo < h2 ? h2 : lo;
  lo = bitonic_clean(a);
  hi = bitonic_clean(b);
}

// The 128-key list's rank r (wave-uniform r < 128).
template <typename T>
__device__ __forceinline__ T rank128(T lo, T hi, int r) {
  return r < kWave ? wbcast(lo, r) : wbcast(hi, r - kWave);
}

// The K (64 < K <= 128) smallest of the wave's E keys per lane, as a sorted
// 128-key list (PAD past the real keys).  The two smallest keys of each lane
// are 128 real keys (or PAD), so their K-th smallest bounds the K-th
// smallest key from above; the keys at or below that bound are sorted at
// once when at most 128, else every key column is merged into the list.
template <int E, typename T>
__device__ void wave_smallest128(const T (&key)[E], int K, T *cbuf, T &lo, T &hi) {
  const T PAD = (T)~(T)0;
  const int lane = lane_id();
  T m1 = PAD, m2 = PAD;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const T v = key[e];
    if (v < m1) {
      m2 = m1;
      m1 = v;
    } else if (v < m2) {
      m2 = v;
    }
  }
  T a, b;
  merge64x2(wsort(m1), wsort(m2), a, b);
  const T tau = rank128(a, b, K - 1);
  int cnt = 0;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool c = key[e] <= tau && key[e] != PAD;
    const uint64_t mk = __ballot(c);
    const int pos = cnt + __popcll(mk & lt);
    if (c && pos < 2 * kWave) cbuf[pos] = key[e];
    cnt += __popcll(mk);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (cnt <= 2 * kWave) {
    merge64x2(wsort(lane < cnt ? cbuf[lane] : PAD), wsort(lane + kWave < cnt ? cbuf[lane + kWave] : PAD), lo, hi);
  } else {
    lo = wsort(key[0]);
    hi = PAD;
#pragma unroll
    for (int e = 1; e < E; ++e) merge128_col(lo, hi, wsort(key[e]));
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();  // cbuf is reused by the next call
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same for N keys get(p), p in [0, N), read twice instead of held in
// registers (64 < K <= 128).
template <typename Get>
__device__ void wave_smallest128_gen(int64_t N, Get get, int K, uint64_t *cbuf, uint64_t &lo, uint64_t &hi) {
  constexpr uint64_t PAD = ~0ull;
  const int lane = lane_id();
  uint64_t m1 = PAD, m2 = PAD;
  for (int64_t p = lane; p < N; p += kWave) {
    const uint64_t v = get(p);
    if (v < m1) {
      m2 = m1;
      m1 = v;
    } else if (v < m2) {
      m2 = v;
    }
  }
  uint64_t a, b;
  merge64x2(wsort(m1), wsort(m2), a, b);
  const uint64_t tau = rank128(a, b, K - 1);
  int cnt = 0;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  for (int64_t p0 = 0; p0 < N; p0 += kWave) {  // wave-uniform trip count
    const int64_t p = p0 + lane;
    const uint64_t v = p < N ? get(p) : PAD;
    const bool c = v <= tau && v != PAD;
    const uint64_t mk = __ballot(c);
    const int pos = cnt + __popcll(mk & lt);
    if (c && pos < 2 * kWave) cbuf[pos] = v;
    cnt += __popcll(mk);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (cnt <= 2 * kWave) {
    merge64x2(wsort(lane < cnt ? cbuf[lane] : PAD), wsort(lane + kWave < cnt ? cbuf[lane + kWave] : PAD), lo, hi);
  } else {
    lo = PAD;
    hi = PAD;
    for (int64_t p0 = 0; p0 < N; p0 += kWave) {
      const int64_t p = p0 + lane;
      merge128_col(lo, hi, wsort(p < N ? get(p) : PAD));
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();  // cbuf is reused by the next call
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same selection on 32-bit keys (PAD = ~0u, above every real key): the
// K smallest come back ascending across the lanes, lane l holding the l-th
// (PAD past the real keys).
template <int E>
__device__ uint32_t wave_smallest_u32(const uint32_t (&key)[E], int K, uint32_t *cbuf) {
  constexpr uint32_t PAD = ~0u;
  const int lane = lane_id();
  uint32_t mn = key[0];
#pragma unroll
  for (int e = 1; e < E; ++e) mn = key[e] < mn ? key[e] : mn;
  const uint32_t tau = (uint32_t)__builtin_amdgcn_readlane((int)wave_sort_u32(mn), K - 1);
  int cnt = 0;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool c = key[e] <= tau && key[e] != PAD;
    const uint64_t mk = __ballot(c);
    const int pos = cnt + __popcll(mk & lt);
    if (c && pos < kWave) cbuf[pos] = key[e];
    cnt += __popcll(mk);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t best;
  if (cnt <= kWave) {
    best = wave_sort_u32(lane < cnt ? cbuf[lane] : PAD);
  } else {
    best = wave_sort_u32(key[0]);
#pragma unroll
    for (int e = 1; e < E; ++e) {
      const uint32_t c = wave_sort_u32(key[e]);
      const uint32_t r = lane_rev_u32(c);  // descending
      uint32_t v = best < r ? best : r;                                // bitonic: the 64 smallest of both
#pragma unroll
      for (int j = kWave / 2; j > 0; j >>= 1) {
        const uint32_t o = lane_xor_u32(v, j);
        v = ((lane & j) == 0) ? (o < v ? o : v) : (o > v ? o : v);
      }
      best = v;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();  // cbuf is reused by the next call
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return best;
}


// Batches that keep their sums point-major (G.flagsets): D[i][s] is the
// running sum S of pair (s, i) (the exact distance once the pair is exact),
// the flags stay slot-major, and the round index is stored only for decided
// and exact pairs -- an undecided sampled pair was sampled up to T[cur].
__device__ __forceinline__ uint8_t pm_round(uint8_t f, uint8_t ri_stored, int cur) {
  return (f & (FL_ACC | FL_DISC | FL_EXACT)) ? ri_stored : (uint8_t)cur;
}

// A slot's round constants, read once into registers (the byte stores of
// the kernels below may alias any object, so the slot would otherwise be
// re-read after each of them).  The bounds are the same expressions as
// point_bounds: d = S / (T W) with T W rounded once, width alpha(T).
struct RoundConsts {
  double TW, a, mW;  // T[cur] W, alpha[cur], m W
};
__device__ __forceinline__ RoundConsts round_consts(const Slot *sl, int64_t m, int cur) {
  RoundConsts rc;
  rc.TW = (double)sl->T[cur] * sl->W;
  rc.a = sl->alpha[cur];
  rc.mW = (double)m * sl->W;
  return rc;
}
// Bounds of a pair: exact (width 0), accepted earlier at round ri, or
// sampled up to T[cur].
__device__ __forceinline__ void pair_bounds(const Slot *sl, const RoundConsts &rc, int64_t S, uint8_t f, uint8_t ri,
                                            bool at_cur, double &d, double &a) {
  if (f & FL_EXACT) {
    d = (double)S / rc.mW;
    a = 0.0;
  } else if (at_cur) {
    d = (double)S / rc.TW;
    a = rc.a;
  } else {
    d = (double)S / ((double)sl->T[ri] * sl->W);
    a = sl->alpha[ri];
  }
}

// Per slot, at the end of its partial-list area, the tiles of this round
// whose kept pairs mix divisors or widths: a count, then the tile indices
// (k_select_pm appends, k_select_pm_mixed selects them, k_select_merge_pm
// clears the count; the first round, which never mixes, starts it at 0).
__host__ __device__ inline int64_t fs_mixed_words(int64_t n) { return ((n + FS_PT - 1) / FS_PT + 2) / 2; }
__device__ __forceinline__ uint32_t *fs_mixed(const Bufs &B, int sl, int64_t n) {
  return reinterpret_cast<uint32_t *>(B.part + (int64_t)(sl + 1) * B.part_stride - fs_mixed_words(n));
}

constexpr int FS_TS = FS_PT + 4;  // LDS row stride in words: rows stay 16-byte aligned

// The sums of a tile of FS_SL slots x FS_PT points, transposed into LDS rows:
// FS_SL / 4 16-byte loads per point (nqp is a multiple of 16), up to four
// points' worth in flight at once per thread (clamped rows, zeroed after).
__device__ __forceinline__ void fs_stage_sums(uint32_t (*t)[FS_TS], const uint32_t *__restrict__ D, int32_t nqp,
                                              int64_t i0, int s0, int64_t n) {
  static_assert(FS_SL % 4 == 0 && FS_SL <= 16, "16-byte pieces of one line per point");
  constexpr int PER = FS_PT / FS_NT, Q = FS_SL / 4, U = PER < 4 ? PER : 4;
#pragma unroll
  for (int u0 = 0; u0 < PER; u0 += U) {
    uint4 v[U][Q];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = min(i0 + threadIdx.x + (u0 + u) * FS_NT, n - 1);
#pragma unroll
      for (int q = 0; q < Q; ++q) v[u][q] = *reinterpret_cast<const uint4 *>(D + i * nqp + s0 + 4 * q);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int pt = threadIdx.x + (u0 + u) * FS_NT;
      const bool in = i0 + pt < n;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        t[4 * q + 0][pt] = in ? v[u][q].x : 0u;
        t[4 * q + 1][pt] = in ? v[u][q].y : 0u;
        t[4 * q + 2][pt] = in ? v[u][q].z : 0u;
        t[4 * q + 3][pt] = in ? v[u][q].w : 0u;
      }
    }
  }
}

// Selection for such batches: one block per tile of FS_SL slots x FS_PT
// points (D transposed through LDS), the tile's k smallest UCB and k+1
// smallest LCB per slot over the kept points (the partial lists that
// k_select_merge_pm reads, one per FS_PT points).  In a sampled round 0 every pair is undecided: its flag and round
// index are initialised here.
// WIDE: some slot's k + 1 exceeds 64 (lists of up to 128 keys; the K <= 64
// instance stays within 64 VGPRs).
template <bool WIDE>
__global__ __launch_bounds__(FS_NT) void k_select_pm(const Slot *__restrict__ slots, const uint32_t *__restrict__ D,
                                                  int32_t nqp, Bufs B, Geometry G, int32_t cur, int32_t init) {
  __shared__ __align__(16) uint32_t t[FS_SL][FS_TS];
  __shared__ uint64_t cbuf[FS_NT / kWave][kWave];
  const int64_t n = G.n, m = G.m;
  const int ns = G.nslots;
  const int64_t ngroups = (nqp + FS_SL - 1) / FS_SL;
  const int64_t nwork = ngroups * ((n + FS_PT - 1) / FS_PT);
  const int64_t w = xcd_work_item(nwork);
  if (w >= nwork) return;
  const int64_t tile = w / ngroups;
  const int64_t i0 = tile * FS_PT;
  const int s0 = (int)(w % ngroups) * FS_SL;
  static_assert(FS_SL == FS_NT / kWave, "one wave per slot of the tile");
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  // this wave's slot, when it runs this round in dense form (wave-uniform);
  // nothing to do unless one of the tile's slots does
  const int sl = s0 + wave;
  const Slot *slp = &slots[sl < ns ? sl : 0];
  const bool act = sl < ns && (slp->state == 1) & (slp->cur == cur) & (slp->implicit != 0);
  if (__syncthreads_or(act ? 1 : 0) == 0) return;
  // whole tile with 4-byte aligned flag rows: each lane takes four runs of
  // four consecutive points (flags as one word, sums as one 16-byte read);
  // the flag words are loaded together with the sums
  const bool fast = i0 + FS_PT <= n && (n & 3) == 0;
  static_assert(FS_E == 16 && FS_PT == 4 * 4 * kWave, "four runs of four points per lane");
  uint8_t *flr = B.fl + (int64_t)(act ? sl : 0) * n + i0;
  uint32_t fpre[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    fpre[u] = (fast && act && !init) ? *reinterpret_cast<const uint32_t *>(flr + 4 * kWave * u + 4 * lane) : 0u;
  fs_stage_sums(t, D, nqp, i0, s0, n);
  __syncthreads();
  constexpr uint32_t PAD32 = ~0u;  // above every sum (S < m * 65025 < 2^32 - 1)
  if (act) {
    const int r = wave;
    const int k = slp->k;
    const RoundConsts rc = round_consts(slp, m, cur);
    // The keys of the kept pairs (their sums; PAD when discarded or past
    // n) and which classes of kept pairs the tile holds: exact, sampled up
    // to T[cur], or accepted in an earlier round.
    uint32_t kt[FS_E];
    bool has_x = false, has_c = false, has_l = false;
    if (fast) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p0 = 4 * kWave * u + 4 * lane;
        const uint32_t fw = fpre[u];
        const uint4 tv = *reinterpret_cast<const uint4 *>(&t[r][p0]);
        constexpr uint32_t ONE = 0x01010101u;
        const uint32_t kept = ~(fw >> 2) & ONE, ex = fw & ONE, ac = (fw >> 1) & ONE;
        has_x |= (kept & ex) != 0;
        has_l |= (kept & ac & ~ex) != 0;
        has_c |= (kept & ~ac & ~ex) != 0;
        kt[4 * u + 0] = (fw & 0x00000004u) ? PAD32 : tv.x;
        kt[4 * u + 1] = (fw & 0x00000400u) ? PAD32 : tv.y;
        kt[4 * u + 2] = (fw & 0x00040000u) ? PAD32 : tv.z;
        kt[4 * u + 3] = (fw & 0x04000000u) ? PAD32 : tv.w;
      }
      if (init) {  // round 0: every pair of the slot is undecided, sampled at round 0
        uint8_t *rir = B.ri + (int64_t)sl * n + i0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int p0 = 4 * kWave * u + 4 * lane;
          *reinterpret_cast<uint32_t *>(flr + p0) = 0u;
          *reinterpret_cast<uint32_t *>(rir + p0) = 0u;
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < FS_E; ++e) {
        const int p = e * kWave + lane;
        const bool in = i0 + p < n;
        const uint8_t f = init ? (uint8_t)(in ? 0 : FL_DISC) : (in ? flr[p] : (uint8_t)FL_DISC);
        const bool kept = !(f & FL_DISC);
        has_x |= kept && (f & FL_EXACT);
        has_l |= kept && (f & FL_ACC) && !(f & FL_EXACT);
        has_c |= kept && !(f & (FL_ACC | FL_EXACT));
        kt[e] = kept ? t[r][p] : PAD32;
      }
      if (init) {
#pragma unroll
        for (int e = 0; e < FS_E; ++e) {
          const int p = e * kWave + lane;
          if (i0 + p < n) {
            flr[p] = 0;
            B.ri[(int64_t)sl * n + i0 + p] = 0;
          }
        }
      }
    }
    // When every kept pair of the tile has the same divisor and width --
    // all sampled up to T[cur] (T W, alpha(T[cur])), or all exact (m W, 0)
    // -- UCB and LCB are both monotone in d^, and d^ is monotone in the
    // integer sum S: the k smallest UCB and the k+1 smallest LCB are
    // d^ + width and d^ - width of the k+1 smallest sums, so one selection
    // on the 32-bit sums serves both lists, with the same values as two
    // separate ones.  Pairs accepted in an earlier round keep their own
    // round's bounds and take the general path.
    const bool any_x = __ballot(has_x) != 0;
    const bool uniform = __ballot(has_l) == 0 && (!any_x || __ballot(has_c) == 0);
    uint64_t *out = B.part + (int64_t)sl * B.part_stride + tile * (2 * k + 1);
    if (uniform) {
      constexpr uint64_t PAD = ~0ull;
      uint32_t bv[2];
      if (!WIDE || k + 1 <= kWave) {
        bv[0] = wave_smallest_u32<FS_E>(kt, k + 1, reinterpret_cast<uint32_t *>(cbuf[wave]));
        bv[1] = PAD32;
      } else {  // (k + 1 <= 128) ranks lane and 64 + lane
        wave_smallest128<FS_E, uint32_t>(kt, k + 1, reinterpret_cast<uint32_t *>(cbuf[wave]), bv[0], bv[1]);
      }
#pragma unroll
      for (int h = 0; h < (WIDE ? 2 : 1); ++h) {
        const int r = lane + kWave * h;
        if (r < k + 1) {
          const uint32_t b = bv[h];
          double d, al;  // the bounds of a pair with sum b, as pair_bounds gives them
          pair_bounds(slp, rc, (int64_t)b, any_x ? (uint8_t)FL_EXACT : (uint8_t)0, (uint8_t)0, true, d, al);
          if (r < k) out[r] = b == PAD32 ? PAD : dkey(d + al);
          out[k + r] = b == PAD32 ? PAD : dkey(d - al);
        }
      }
    }
    if (lane == 0) {
      uint32_t *ml = fs_mixed(B, sl, n);
      if (init && tile == 0) ml[0] = 0;  // (round 0 never mixes: no appends race with this)
      if (!uniform) ml[1 + atomicAdd(&ml[0], 1u)] = (uint32_t)tile;  // k_select_pm_mixed selects it
    }
  }
}

// The tiles that k_select_pm listed as mixed (pairs exact, sampled at the
// round and accepted in earlier rounds side by side): each kept pair's
// bounds from its own flag and round, then the k smallest UCB and the k+1
// smallest LCB.  One single-wave block per slot; a slot without such tiles
// leaves at once.
__global__ __launch_bounds__(kWave) void k_select_pm_mixed(const Slot *__restrict__ slots,
                                                           const uint32_t *__restrict__ D, int32_t nqp, Bufs B,
                                                           Geometry G, int32_t cur, int32_t init) {
  __shared__ uint32_t tc[FS_PT];
  __shared__ uint64_t cbuf[2 * kWave];
  const int64_t n = G.n, m = G.m;
  const int sl = blockIdx.x;
  if (init || sl >= G.nslots) return;
  const Slot *slp = &slots[sl];
  if (slp->state != 1 || slp->cur != cur || slp->implicit == 0) return;
  const uint32_t *ml = fs_mixed(B, sl, n);
  const uint32_t nmix = ml[0];
  const int lane = lane_id();
  const int k = slp->k;
  const RoundConsts rc = round_consts(slp, m, cur);
  for (uint32_t e0 = 0; e0 < nmix; ++e0) {
    const int64_t tile = ml[1 + e0];
    const int64_t i0 = tile * FS_PT;
    __builtin_amdgcn_s_barrier();  // (one wave) the previous tile's reads of tc are done
#pragma unroll
    for (int e = 0; e < FS_E; ++e) {  // this slot's column of the tile (a rare path: 4-byte loads)
      const int p = e * kWave + lane;
      tc[p] = i0 + p < n ? D[(i0 + p) * nqp + sl] : 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint8_t *flr = B.fl + (int64_t)sl * n + i0;
    uint64_t *out = B.part + (int64_t)sl * B.part_stride + tile * (2 * k + 1);
    // upper bounds, then lower bounds: one key array live at a time
#pragma nounroll
    for (int lower = 0; lower < 2; ++lower) {
      uint64_t key[FS_E];
#pragma unroll
      for (int e = 0; e < FS_E; ++e) {
        const int p = e * kWave + lane;
        const int64_t i = i0 + p;
        key[e] = ~0ull;
        if (i >= n) continue;
        const uint8_t f = flr[p];
        if (f & FL_DISC) continue;
        const bool late = (f & FL_ACC) && !(f & FL_EXACT);  // accepted before this round
        double d, al;
        pair_bounds(slp, rc, (int64_t)tc[p], f, late ? B.ri[(int64_t)sl * n + i] : (uint8_t)0, !late, d, al);
        key[e] = lower ? dkey(d - al) : dkey(d + al);
      }
      const int K = lower ? k + 1 : k;
      uint64_t *o = lower ? out + k : out;
      if (K <= kWave) {
        wave_smallest<FS_E>(key, K, o, cbuf);
      } else {  // (K <= 128)
        uint64_t lo, hi;
        wave_smallest128<FS_E, uint64_t>(key, K, cbuf, lo, hi);
        o[lane] = lo;
        if (lane + kWave < K) o[lane + kWave] = hi;
      }
    }
  }
}

// Decide for such batches, per tile of DQ_SL slots x DQ_PT points: the
// slot-major flags are staged in LDS as one word per (group of four slots,
// point), each thread keeps its group's thresholds in registers and decides
// the group's four pairs of a point at once from D read point-major, writes
// the next round's point-major "not sampled" bytes A, and the changed flags
// (and the round index of pairs decided while sampled) go back slot-major.
// Per slot the tile's counts of undecided sampled, undecided exact and newly
// accepted pairs go to the slot's partial-list area (consumed by k_finish),
// so no atomics are needed.
constexpr int DQ_SL = 64, DQ_PT = 512;
constexpr int DQ_G = DQ_SL / 4;   // groups of four slots
constexpr int DQ_TS = DQ_PT + 4;  // LDS row stride in words
__global__ __launch_bounds__(NT) void k_decide_pm(Slot *__restrict__ slots, const uint32_t *__restrict__ D,
                                                  uint8_t *__restrict__ A, int32_t nqp, Bufs B, Geometry G,
                                                  int32_t cur) {
  // ft[g][p]: byte j holds the flag of slot s0 + 4 g + j at point i0 + p.
  // The row stride (DQ_PT + 4 words) puts the 16 groups x 4 points that a
  // wave reads at once in different banks.
  __shared__ __align__(16) uint32_t ft[DQ_G][DQ_TS];
  const int64_t n = G.n;
  const int ns = G.nslots;
  const int64_t ngroups = (nqp + DQ_SL - 1) / DQ_SL;
  const int64_t nwork = ngroups * ((n + DQ_PT - 1) / DQ_PT);
  const int64_t w = xcd_work_item(nwork);
  if (w >= nwork) return;
  const int64_t tile = w / ngroups;
  const int64_t i0 = tile * DQ_PT;
  const int s0 = (int)(w % ngroups) * DQ_SL;
  const int pts = (int)min((int64_t)DQ_PT, n - i0);
  // which slots of the tile run this round (one read per slot, in parallel)
  __shared__ uint8_t srun[DQ_SL];
  __shared__ int sany;
  if (threadIdx.x == 0) sany = 0;
  __syncthreads();
  if (threadIdx.x < DQ_SL) {
    const int sl = s0 + threadIdx.x;
    srun[threadIdx.x] =
        (sl < ns && slots[sl].state == 1 && slots[sl].cur == cur && slots[sl].implicit != 0) ? 1 : 0;
    if (srun[threadIdx.x]) sany = 1;
  }
  __syncthreads();
  if (!sany) return;  // every slot of the tile is idle or sparse
  static_assert(FL_EXACT == 1 && FL_ACC == 2 && FL_DISC == 4, "flag bits 0, 1, 2; bit 7 marks a change");
  // stage the flags of the running slots (others: discarded, "not sampled")
  if ((n & 3) == 0 && pts == DQ_PT) {
    // whole tile, 4-byte words: each thread reads the same word (four
    // points) of its group's four rows -- the lanes of a wave take
    // consecutive words of one row -- and writes the four points' words,
    // the 4 x 4 bytes transposed
    constexpr int QW = DQ_PT / 4, ITEMS = DQ_G * QW / NT;
    static_assert(DQ_G * QW % NT == 0 && QW % kWave == 0, "whole items per thread, one group per wave load");
    uint32_t wv[ITEMS][4];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int idx = threadIdx.x + it * NT, g = idx / QW, c = idx % QW;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * g + j;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(B.fl + (int64_t)(srun[r] ? s0 + r : 0) * n + i0);
        wv[it][j] = srun[r] ? src[c] : 0x04040404u;
      }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int idx = threadIdx.x + it * NT, g = idx / QW, c = idx % QW;
      uint32_t o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        o[e] = ((wv[it][0] >> (8 * e)) & 0xFFu) | (((wv[it][1] >> (8 * e)) & 0xFFu) << 8) |
               (((wv[it][2] >> (8 * e)) & 0xFFu) << 16) | (((wv[it][3] >> (8 * e)) & 0xFFu) << 24);
      *reinterpret_cast<uint4 *>(&ft[g][4 * c]) = make_uint4(o[0], o[1], o[2], o[3]);
    }
  } else {
    for (int r = threadIdx.x / kWave; r < DQ_SL; r += NT / kWave) {
      const bool run = srun[r] != 0;
      const uint8_t *src = B.fl + (int64_t)(run ? s0 + r : 0) * n + i0;
      uint8_t *dst = reinterpret_cast<uint8_t *>(&ft[r >> 2][0]) + (r & 3);
      for (int p = lane_id(); p < DQ_PT; p += kWave) dst[4 * p] = (run && p < pts) ? src[p] : (uint8_t)FL_DISC;
    }
  }
  __syncthreads();
  // Each thread takes one group of four consecutive slots (one 16-byte
  // load of their sums, one flag word and one 4-byte store of their "not
  // sampled" bytes per point; nqp is a multiple of 16) and every DQ_P-th
  // point.  Per-slot counts are kept as bytes of one word (at most
  // DQ_PT / DQ_P = 32 per thread, 128 after the sum over a wave's four
  // threads of a group).
  constexpr int DQ_P = NT / DQ_G;
  static_assert(NT % DQ_G == 0 && DQ_PT / DQ_P * (kWave / DQ_G) < 256, "byte counters");
  __shared__ int cnt[NT / kWave][DQ_SL][3];
  const int g = threadIdx.x % DQ_G, c4 = 4 * g;  // this thread's group; its first slot within the tile
  uint32_t runm = 0;  // bit 0 of byte j: slot c4 + j runs
#pragma unroll
  for (int j = 0; j < 4; ++j) runm |= (srun[c4 + j] ? 1u : 0u) << (8 * j);
  uint32_t c_act = 0, c_xa = 0, c_acc = 0;  // byte j: slot c4 + j
  if (s0 + c4 < nqp) {
    // the decisions as thresholds on the sums (k_select_merge_pm derives them
    // from U, L1, L2 with the FP64 bounds), so no pair needs a division.  A
    // threshold t in [-1, 2^32) becomes the 32-bit bound min(max(t + 1, 0),
    // 2^32 - 1): with every sum below 2^32 - 1, S > t holds exactly when
    // S >= bound, and S <= t exactly when S < bound.
    auto bound = [](int64_t t) -> uint32_t {
      return t + 1 <= 0 ? 0u : (t + 1 >= 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)(t + 1));
    };
    // (named fields, picked by arithmetic below: a select between two array
    // elements would become an indexed load from scratch memory)
    struct Thr {
      uint32_t disc, acc, xdisc, xacc;  // discard: S >= disc; accept: S < acc (sampled / exact pairs)
    } th[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool rj = (runm >> (8 * j)) & 1u;
      const Slot &sj = slots[rj ? s0 + c4 + j : 0];
      th[j].disc = rj ? bound(sj.sthr[0]) : 0u;
      th[j].acc = rj ? bound(sj.sthr[1]) : 0u;
      th[j].xdisc = rj ? bound(sj.sthr[2]) : 0u;
      th[j].xacc = rj ? bound(sj.sthr[3]) : 0u;
    }
    // DQ_B points per batch: their sums are loaded together, so the loads'
    // latency is paid once per batch
    constexpr int DQ_B = 4;
    uint4 sn[DQ_B];  // the next batch's sums, loaded while the current batch is decided
    auto load_batch = [&](int pb, uint4 (&sv)[DQ_B]) {
#pragma unroll
      for (int b = 0; b < DQ_B; ++b) {  // unconditional loads (clamped to the tile): all in flight at once
        const int p = min(pb + b * DQ_P, pts - 1);
        sv[b] = *reinterpret_cast<const uint4 *>(D + (i0 + p) * nqp + s0 + c4);
      }
    };
    constexpr uint32_t B0 = 0x01010101u;
    load_batch(threadIdx.x / DQ_G, sn);
    for (int pb = threadIdx.x / DQ_G; pb < pts; pb += DQ_P * DQ_B) {
      uint4 sv[DQ_B];
#pragma unroll
      for (int b = 0; b < DQ_B; ++b) sv[b] = sn[b];
      if (pb + DQ_P * DQ_B < pts) load_batch(pb + DQ_P * DQ_B, sn);
#pragma unroll
      for (int b = 0; b < DQ_B; ++b) {
        const int p = pb + b * DQ_P;
        if (p >= pts) break;
        uint32_t f = ft[g][p];
        // bit 0 of byte j: the pair is undecided (running, neither accepted nor discarded)
        const uint32_t und = runm & ~((f >> 1) | (f >> 2)) & B0;
        if (und) {
          const uint32_t S4[4] = {sv[b].x, sv[b].y, sv[b].z, sv[b].w};
          uint32_t dm = 0, am = 0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t xm = 0u - ((f >> (8 * j)) & 1u);  // all ones for an exact pair
            const uint32_t td = th[j].disc ^ ((th[j].disc ^ th[j].xdisc) & xm);
            const uint32_t ta = th[j].acc ^ ((th[j].acc ^ th[j].xacc) & xm);
            const bool dj = S4[j] >= td;
            dm |= (dj ? 1u : 0u) << (8 * j);
            am |= ((!dj && S4[j] < ta) ? 1u : 0u) << (8 * j);
          }
          dm &= und;
          am &= und;
          const uint32_t rest = und & ~dm & ~am, ex = f & B0;
          c_acc += am;
          c_xa += rest & ex;
          c_act += rest & ~ex;
          if (dm | am) {
            f |= (dm << 2) | (am << 1) | ((dm | am) << 7);
            ft[g][p] = f;
          }
        }
        // "not sampled" next round: not running, or any flag set (bits 0..6)
        const uint32_t nz = (((f & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) >> 7) & B0;
        *reinterpret_cast<uint32_t *>(A + (i0 + p) * nqp + s0 + c4) = nz | (~runm & B0);
      }
    }
  }
  // per wave, the lanes with the same group (DQ_G apart) add their counts
  static_assert(kWave == 4 * DQ_G, "four lanes of a wave share a slot group");
#pragma unroll
  for (int o = DQ_G; o < kWave; o <<= 1) {
    c_act += (uint32_t)__shfl_xor((int)c_act, o);
    c_xa += (uint32_t)__shfl_xor((int)c_xa, o);
    c_acc += (uint32_t)__shfl_xor((int)c_acc, o);
  }
  if (lane_id() < DQ_G) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cnt[threadIdx.x / kWave][c4 + j][0] = (int)((c_act >> (8 * j)) & 0xFFu);
      cnt[threadIdx.x / kWave][c4 + j][1] = (int)((c_xa >> (8 * j)) & 0xFFu);
      cnt[threadIdx.x / kWave][c4 + j][2] = (int)((c_acc >> (8 * j)) & 0xFFu);
    }
  }
  __syncthreads();
  if (threadIdx.x < DQ_SL && srun[threadIdx.x]) {
    const int cs = threadIdx.x;
    const int s = s0 + cs;
    {
      int tot[3] = {0, 0, 0};
      for (int q = 0; q < NT / kWave; ++q)
        for (int k = 0; k < 3; ++k) tot[k] += cnt[q][cs][k];
      uint32_t *rec = reinterpret_cast<uint32_t *>(B.part + (int64_t)s * B.part_stride) + 3 * tile;
      rec[0] = (uint32_t)tot[0];
      rec[1] = (uint32_t)tot[1];
      rec[2] = (uint32_t)tot[2];
    }
  }
  // changed flags back, slot-major; a pair decided while still sampled
  // records the round of its last samples
  for (int r = threadIdx.x / kWave; r < DQ_SL; r += NT / kWave) {
    const int s = s0 + r;
    if (s >= ns) break;
    const uint8_t *row = reinterpret_cast<const uint8_t *>(&ft[r >> 2][0]) + (r & 3);
    for (int p = lane_id(); p < pts; p += kWave) {
      const uint8_t f = row[4 * p];
      if (!(f & 0x80)) continue;
      const int64_t off = (int64_t)s * n + i0 + p;
      B.fl[off] = f & 0x7F;
      if (!(f & FL_EXACT)) B.ri[off] = (uint8_t)cur;
    }
  }
}

constexpr int MT = 1024;  // merge / finish block size

// The decisions of an undecided pair at the current round as integer
// thresholds on its sum S.  d = S / (T W) (or S / (m W) once exact) is a
// correctly rounded quotient of an exactly represented integer, hence
// non-decreasing in S, and so are UCB and LCB: "not discarded" (LCB <= U)
// and "accepted" (UCB <= L2, or d <= L1 for an exact pair) hold exactly for
// the sums up to some threshold.  The threshold is searched over [-1, 2^32)
// with the same FP64 expressions as every other decision (kind 0/1:
// keep/accept of a sampled pair, 2/3: of an exact pair); -1 means no sum
// qualifies.  Sixteen lanes of a wave search one threshold together: each
// step tests sixteen sums spread over the open interval and keeps the part
// between the last one that holds and the first one that fails (the
// decisions are monotone in the sum, so those that hold come first), about
// eight steps instead of thirty-three halvings.  Lanes 16 j .. 16 j + 15
// return threshold j (a whole wave calls it).
__device__ int64_t sum_threshold_wave(const Slot *sl, const RoundConsts &rc, double U, double L1, double L2) {
  const int lane = lane_id(), kind = lane >> 4, sub = lane & 15;
  const bool exact = kind >= 2, accept = (kind & 1) != 0;
  auto holds = [&](int64_t S) -> bool {
    double d, al;
    pair_bounds(sl, rc, S, exact ? (uint8_t)FL_EXACT : (uint8_t)0, (uint8_t)0, true, d, al);
    const double ucb = d + al, lcb = d - al;
    if (!accept) return !(lcb > U);
    return exact ? (ucb <= L1) : (ucb <= L2);
  };
  int64_t lo = -1, hi = (int64_t)1 << 32;  // holds at lo (or lo = -1), fails at hi (or hi = 2^32)
  // (lo and hi are the same in the sixteen lanes of a group: the loop is
  // group-uniform, and the ballot and shuffles read lanes of the own group)
  while (hi - lo > 1) {
    const int64_t probe = lo + ((hi - lo) * (sub + 1)) / 17;  // in (lo, hi), ascending in sub
    const bool h = holds(probe);
    const uint32_t mask = (uint32_t)(__ballot(h) >> (16 * kind)) & 0xFFFFu;
    const int c = __popc(mask);  // the probes that hold: sub < c
    const int64_t plo = shfl_i64(probe, 16 * kind + (c > 0 ? c - 1 : 0));
    const int64_t phi = shfl_i64(probe, 16 * kind + (c < 16 ? c : 15));
    if (c > 0) lo = plo;
    if (c < 16) hi = phi;
  }
  return lo;
}

// U, L1, L2 from the partial lists of k_select_partial (one per SEL_CH
// elements of P).  skip_dense: the dense slots of a point-major batch are
// k_select_merge_pm's.
__global__ __launch_bounds__(MT) void k_select_merge(Slot *__restrict__ slots, Bufs B, Geometry G, int32_t skip_dense) {
  const int s = blockIdx.x;
  Slot *sl = &slots[s];
  if (sl->state != 1) return;
  if (skip_dense && sl->implicit != 0) return;
  const int64_t nP = size_P(sl, G.n);
  const int64_t nch = (nP + SEL_CH - 1) / SEL_CH;
  const int k = sl->k;
  const int64_t w = 2 * k + 1;
  const uint64_t *part = B.part + (int64_t)s * B.part_stride;
  __shared__ SelScratch ss;
  int less;
  auto gu = [&](int64_t p) -> uint64_t { return part[(p / k) * w + (p % k)]; };
  auto gl = [&](int64_t p) -> uint64_t { return part[(p / (k + 1)) * w + k + (p % (k + 1))]; };
  const uint64_t U = block_kth_gen<MT>(nch * k, gu, k, ss, &less);
  const uint64_t L1 = block_kth_gen<MT>(nch * (k + 1), gl, k, ss, &less);
  const uint64_t L2 = block_kth_gen<MT>(nch * (k + 1), gl, k + 1, ss, &less);
  if (threadIdx.x == 0) {
    sl->U = dkey_inv(U);
    sl->L1 = dkey_inv(L1);
    sl->L2 = dkey_inv(L2);
  }
}

// The same for the dense slots of a point-major batch over the partial
// lists of k_select_pm (one per FS_PT points of [0, n)): one block of two
// waves per slot, the first selecting U and the second L1 and L2 at the same
// time; then the decisions as thresholds on the sums, for k_decide_pm.
constexpr int SMP_T = 2 * kWave;
__global__ __launch_bounds__(SMP_T) void k_select_merge_pm(Slot *__restrict__ slots, Bufs B, Geometry G) {
  __shared__ uint64_t cbuf[2][2 * kWave];
  __shared__ uint64_t ul[3];  // U, L1, L2 as keys
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int s = blockIdx.x;
  if (s >= G.nslots) return;  // block-uniform from here on
  Slot *sl = &slots[s];
  if (sl->state != 1 || sl->implicit == 0) return;
  const int64_t nch = (G.n + FS_PT - 1) / FS_PT;
  const int k = sl->k;
  const int64_t w = 2 * k + 1;
  const uint64_t *part = B.part + (int64_t)s * B.part_stride;
  // (32-bit index arithmetic: the lists hold fewer than 2^32 keys)
  const uint32_t ku = (uint32_t)k, kl = (uint32_t)k + 1u, wu = (uint32_t)w;
  if (wave == 0) {
    auto gu = [&](int64_t p) -> uint64_t {
      const uint32_t q = (uint32_t)p / ku;
      return part[q * wu + ((uint32_t)p - q * ku)];
    };
    uint64_t U;
    if (k <= kWave) {
      U = wave_bcast_u64(wave_smallest_gen(nch * k, gu, k, cbuf[0]), k - 1);
    } else {
      uint64_t lo, hi;
      wave_smallest128_gen(nch * k, gu, k, cbuf[0], lo, hi);
      U = rank128(lo, hi, k - 1);
    }
    if (lane == 0) ul[0] = U;
  } else {
    auto gl = [&](int64_t p) -> uint64_t {
      const uint32_t q = (uint32_t)p / kl;
      return part[q * wu + ku + ((uint32_t)p - q * kl)];
    };
    uint64_t L1, L2;
    if (k + 1 <= kWave) {
      const uint64_t lcb = wave_smallest_gen(nch * (k + 1), gl, k + 1, cbuf[1]);
      L1 = wave_bcast_u64(lcb, k - 1);
      L2 = wave_bcast_u64(lcb, k);
    } else {
      uint64_t lo, hi;
      wave_smallest128_gen(nch * (k + 1), gl, k + 1, cbuf[1], lo, hi);
      L1 = rank128(lo, hi, k - 1);
      L2 = rank128(lo, hi, k);
    }
    if (lane == 0) {
      ul[1] = L1;
      ul[2] = L2;
    }
  }
  __syncthreads();
  if (wave != 0) return;
  const double U = dkey_inv(ul[0]), L1 = dkey_inv(ul[1]), L2 = dkey_inv(ul[2]);
  if (lane == 0) {
    sl->U = U;
    sl->L1 = L1;
    sl->L2 = L2;
  }
  const RoundConsts rc = round_consts(sl, G.m, sl->cur);
  const int64_t thr = sum_threshold_wave(sl, rc, U, L1, L2);
  if ((lane & 15) == 0) sl->sthr[lane >> 4] = thr;
  if (lane == 0) fs_mixed(B, s, G.n)[0] = 0;  // the next round's list of mixed tiles starts empty
}

// ---------------------------------------------------------------- decide

constexpr int DEC_E = 8;
constexpr int DEC_CH = NT * DEC_E;

// Discard if LCB > U (k kept points are surely closer); accept if fewer
// than k other points can be closer (UCB <= L2, or for an exact point
// d <= L1); otherwise keep undecided.  Survivors are compacted into the
// next lists with one atomic per list and block (ballots give each lane its
// place); order within a list is irrelevant to the result.
__device__ void decide_chunk(Slot *sl, int s, int64_t chunk, int64_t nA, const Bufs &B, const Geometry &G) {
  const int64_t n = G.n, m = G.m;
  const int64_t base = chunk * DEC_CH;
  const SlotArrays a = slot_arrays(B, n, s, sl->par);
  const double U = sl->U, L1 = sl->L1, L2 = sl->L2;
  constexpr int NW = NT / kWave;
  __shared__ int wcnt[DEC_E][NW][3];
  __shared__ int bbase[3];
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  int cat[DEC_E];  // 0 act, 1 xa, 2 acc, -1 none
  int32_t id[DEC_E];
#pragma unroll
  for (int e = 0; e < DEC_E; ++e) {
    const int64_t p = base + (int64_t)e * NT + threadIdx.x;
    cat[e] = -1;
    id[e] = 0;
    if (p < nA) {
      const int32_t i = elem_A(sl, a, p);
      id[e] = i;
      const uint8_t f = a.fl[i];
      double d, al;
      point_bounds(sl, m, a.S[i], f, a.ri[i], d, al);
      const double ucb = d + al, lcb = d - al;
      const bool exact = (f & FL_EXACT) != 0;
      if (lcb > U) {
        a.fl[i] = f | FL_DISC;
      } else if (exact ? (ucb <= L1) : (ucb <= L2)) {
        a.fl[i] = f | FL_ACC;
        cat[e] = 2;
      } else {
        cat[e] = exact ? 1 : 0;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < DEC_E; ++e) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint64_t mk = __ballot(cat[e] == c);
      if (lane == 0) wcnt[e][wave][c] = __popcll(mk);
    }
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int c = threadIdx.x;
    int tot = 0;
    for (int e = 0; e < DEC_E; ++e)
      for (int w = 0; w < NW; ++w) {
        const int t = wcnt[e][w][c];
        wcnt[e][w][c] = tot;  // exclusive prefix in (e, wave) order
        tot += t;
      }
    int *ctr = c == 0 ? &sl->nn_act : (c == 1 ? &sl->nn_xa : &sl->nn_acc);
    bbase[c] = tot ? atomicAdd(ctr, tot) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < DEC_E; ++e) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint64_t mk = __ballot(cat[e] == c);
      if (cat[e] == c) {
        const int pos = bbase[c] + wcnt[e][wave][c] + __popcll(mk & lt_mask);
        int32_t *dst = c == 0 ? a.act_n : (c == 1 ? a.xa_n : a.acc);
        dst[pos] = id[e];
      }
    }
  }
}

// Chunks blockIdx.x, blockIdx.x + gridDim.x, ... of the slot's undecided list.
__global__ __launch_bounds__(NT) void k_decide(Slot *__restrict__ slots, Bufs B, Geometry G) {
  const int s = blockIdx.y;
  Slot *sl = &slots[s];
  if (sl->state != 1) return;
  if (G.flagsets && sl->implicit != 0) return;  // a dense slot of a point-major batch
  const int64_t nA = size_A(sl, G.n);
  for (int64_t c = blockIdx.x; c * DEC_CH < nA; c += gridDim.x) {
    decide_chunk(sl, s, c, nA, B, G);
    __syncthreads();  // the next chunk reuses the block's LDS
  }
}

// ---------------------------------------------------------------- candidate-exact

constexpr int CAND_E = 16;
constexpr int CAND_CH = NT * CAND_E;

// Per chunk of the undecided set: the c_exact smallest (estimate, index).
__global__ __launch_bounds__(NT) void k_cand_partial(Slot *__restrict__ slots, Bufs B, Geometry G) {
  const int s = blockIdx.y;
  const Slot *sl = &slots[s];
  if (sl->state != 1 || sl->c_exact <= 0) return;
  const int64_t n = G.n, m = G.m;
  const int64_t nA = size_A(sl, n);
  const int64_t base = (int64_t)blockIdx.x * CAND_CH;
  if (base >= nA) return;
  const SlotArrays a = slot_arrays(B, n, s, sl->par);
  const int c = min(sl->c_exact, CAND_CH);
  __shared__ SelScratch ss;
  __shared__ int cnt;
  uint64_t key[CAND_E];
  uint32_t id[CAND_E];
#pragma unroll
  for (int e = 0; e < CAND_E; ++e) {
    const int64_t p = base + (int64_t)e * NT + threadIdx.x;
    if (p < nA) {
      const int32_t i = elem_A(sl, a, p);
      double d, al;
      point_bounds(sl, m, a.S[i], a.fl[i], a.ri[i], d, al);
      key[e] = dkey(d);
      id[e] = (uint32_t)i;
    } else {
      key[e] = ~0ull;
      id[e] = 0xFFFFFFFFu;
    }
  }
  int less;
  const uint64_t v = block_kth_regs<NT, CAND_E>(key, c, ss, &less);
  const int need = c - less;
  // index tie-break among keys equal to v
  uint32_t prefix = 0, mask = 0;
  int r = need;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += NT) ss.hist[b] = 0;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < CAND_E; ++e)
      if (key[e] == v && (id[e] & mask) == prefix) atomicAdd(&ss.hist[(id[e] >> shift) & 255u], 1u);
    __syncthreads();
    if (threadIdx.x < kWave) scan_find_bucket(ss, r);
    __syncthreads();
    r -= ss.res[1];
    prefix |= (uint32_t)ss.res[0] << shift;
    mask |= 0xFFu << shift;
    __syncthreads();
  }
  const uint32_t idthr = prefix;
  uint64_t *ok = B.part + (int64_t)s * B.part_stride + (int64_t)blockIdx.x * c;
  const int64_t nchA = (nA + CAND_CH - 1) / CAND_CH;
  uint32_t *oi = reinterpret_cast<uint32_t *>(B.part + (int64_t)s * B.part_stride + nchA * c) +
                 (int64_t)blockIdx.x * c;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
#pragma unroll
  for (int e = 0; e < CAND_E; ++e) {
    if (key[e] < v || (key[e] == v && id[e] <= idthr)) {
      const int pos = atomicAdd(&cnt, 1);
      if (pos < c) {
        ok[pos] = key[e];
        oi[pos] = id[e];
      }
    }
  }
  __syncthreads();
}

template <int DT>
__global__ __launch_bounds__(MT) void k_cand_merge(Slot *__restrict__ slots, const uint8_t *__restrict__ X,
                                                   Bufs B, Geometry G) {
  const int s = blockIdx.x;
  Slot *sl = &slots[s];
  if (sl->state != 1 || sl->c_exact <= 0) return;
  const int64_t n = G.n, m = G.m;
  const int64_t nA = size_A(sl, n);
  const int64_t nchA = (nA + CAND_CH - 1) / CAND_CH;
  const int c = min(sl->c_exact, CAND_CH);
  const int64_t N = nchA * c;
  const uint64_t *pk = B.part + (int64_t)s * B.part_stride;
  const uint32_t *pi = reinterpret_cast<const uint32_t *>(pk + nchA * c);
  const SlotArrays a = slot_arrays(B, n, s, sl->par);
  __shared__ SelScratch ss;
  __shared__ int cnt;
  __shared__ int32_t pick[kMaxKH];
  __shared__ int64_t red[MT / kWave];
  const int take = (int)min((int64_t)c, nA);
  int less;
  const uint64_t v = block_kth_gen<MT>(N, [&](int64_t p) { return pk[p]; }, take, ss, &less);
  const uint32_t thr = block_kth_u32_gen<MT>(
      N, [&](int64_t p) { return pi[p]; }, [&](int64_t p) { return pk[p] == v; }, take - less, ss);
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int64_t p = threadIdx.x; p < N; p += MT) {
    const uint64_t kk = pk[p];
    if (kk == ~0ull) continue;
    if (kk < v || (kk == v && pi[p] <= thr)) {
      const int pos = atomicAdd(&cnt, 1);
      if (pos < kMaxKH) pick[pos] = (int32_t)pi[p];
    }
  }
  __syncthreads();
  const int np = min(cnt, take);
  const int F = sl->F;
  const uint8_t *q = reinterpret_cast<const uint8_t *>(sl->q);
  int64_t made = 0, cost = 0;
  for (int t = 0; t < np; ++t) {
    const int32_t i = pick[t];
    if (a.fl[i] & FL_EXACT) continue;
    // m coordinates, or the m - T not yet sampled without replacement
    cost += sl->norepl ? m - (int64_t)sl->T[a.ri[i]] : m;
    const int64_t tot = block_exact_sum<DT, MT>(X, m, i, q, F, G.metric, red);
    if (threadIdx.x == 0) {
      a.S[i] = tot;
      a.fl[i] = a.fl[i] | FL_EXACT;
    }
    ++made;
    __syncthreads();
  }
  if (threadIdx.x == 0 && made) {
    sl->exact_points += made;
    sl->coord_evals += cost;
  }
}

// ---------------------------------------------------------------- finish

__device__ void write_trivial(const QDesc &qd, int64_t n) {
  const int64_t cnt = qd.kh < n ? qd.kh : n;
  for (int64_t j = threadIdx.x; j < qd.out_stride; j += blockDim.x) qd.out_idx[j] = j < cnt ? j : -1;
  if (threadIdx.x == 0) {
    *qd.out_count = (int32_t)cnt;
    if (qd.out_stats) {
      qd.out_stats->coord_evals = 0;
      qd.out_stats->rounds = 0;
      qd.out_stats->count = (int32_t)cnt;
      qd.out_stats->exact_points = 0;
    }
  }
}

// Output: the kept set ordered by (estimate, index), at most k+h entries.
// An oversized stop (no undecided point left to sample, |P| > k+h) first
// makes the remaining estimated points exact, then keeps the k+h smallest
// by (distance, index), which contain a k-NN set also under ties.
// Slots that keep no lists (implicit 2): builds act / xa / acc from the
// flags (undecided sampled, undecided exact, accepted; discarded points
// dropped) and switches the slot to list mode.  Each wave places its points
// in index order within a range that one LDS atomic per class reserves, so
// the lists are in no particular order overall (no consumer depends on it:
// the decide step compacts its lists the same way), and a wave with no kept
// point does no scan.  With the sums kept point-major, the listed points'
// sums and round indices are copied into the slot-major arrays that the
// list kernels read (with `all`, the sums of the discarded points too, so
// the slot-major state is whole).
// all: for a slot that turns sparse (every undecided point listed, the
// sums copied by k_pm_to_slot afterwards); otherwise the kept points' sums
// are copied here (a finishing slot).
__device__ void lists_from_flags(Slot *sl, int s, const Bufs &B, const Geometry &G, bool all = false) {
  const int64_t n = G.n;
  const SlotArrays a = slot_arrays(B, n, s, sl->par);
  constexpr int V = 16;  // V consecutive points per thread and pass
  __shared__ int run[3];
  const int lane = lane_id();
  const bool vec = (n % V) == 0;  // the slot's flag row is 16-byte aligned
  if (threadIdx.x < 3) run[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t b = 0; b < n; b += (int64_t)MT * V) {
    const int64_t i0 = b + (int64_t)threadIdx.x * V;
    uint8_t f[V];
    if (vec && i0 + V <= n) {
      const uint4 w = *reinterpret_cast<const uint4 *>(a.fl + i0);
      const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int v = 0; v < V; ++v) f[v] = (uint8_t)(ww[v >> 2] >> (8 * (v & 3)));
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) f[v] = i0 + v < n ? a.fl[i0 + v] : (uint8_t)FL_DISC;
    }
    // class of each point: -1 discarded, 0 undecided sampled, 1 undecided exact, 2 accepted
    int c3[3] = {0, 0, 0};
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const uint8_t g = f[v];
      if (g & FL_DISC) continue;
      ++c3[(g & FL_ACC) ? 2 : (g & FL_EXACT) ? 1 : 0];
    }
    int pos[3] = {0, 0, 0};
    if (__ballot(c3[0] + c3[1] + c3[2] > 0) != 0) {  // (wave-uniform)
      // inclusive scan over the wave's lanes, then the wave's range
      int inc[3] = {c3[0], c3[1], c3[2]};
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int t = __shfl_up(inc[k], d);
          if (lane >= d) inc[k] += t;
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        int base = 0;
        if (lane == kWave - 1 && inc[k] > 0) base = atomicAdd(&run[k], inc[k]);
        pos[k] = __shfl(base, kWave - 1) + inc[k] - c3[k];
      }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int64_t i = i0 + v;
      const uint8_t g = f[v];
      const int c = (g & FL_DISC) ? -1 : (g & FL_ACC) ? 2 : (g & FL_EXACT) ? 1 : 0;
      if (c >= 0) {
        int32_t *dst = c == 0 ? a.act : (c == 1 ? a.xa : a.acc);
        dst[pos[c]++] = (int32_t)i;
        if (c == 0 && G.flagsets) a.ri[i] = (uint8_t)sl->cur;
      }
      if (G.flagsets && i < n && c >= 0 && !all) a.S[i] = (int64_t)B.dpm[i * B.dpm_stride + s];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sl->n_act = run[0];
    sl->n_xa = run[1];
    sl->n_acc = run[2];
    sl->implicit = 0;
    if (all && G.flagsets) sl->pm_copy = 1;
  }
  __syncthreads();
}

// The step's slots that turned sparse (pm_copy) take their running sums
// slot-major: S[s][i] = D[i][s] for every point, 64 x 64 tiles transposed
// through LDS so that the point-major reads and slot-major writes are both
// coalesced.  Tiles whose 64 slots have nothing to copy leave at once.
__global__ __launch_bounds__(NT) void k_pm_to_slot(const Slot *__restrict__ slots, const uint32_t *__restrict__ D,
                                                   int32_t nqp, Bufs B, Geometry G) {
  __shared__ uint32_t t[FT][FT + 1];
  __shared__ uint8_t cp[FT];
  __shared__ int any;
  const int64_t n = G.n;
  const int ns = G.nslots;
  const int s0 = (int)blockIdx.y * FT;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (threadIdx.x < FT) {
    const int sl = s0 + threadIdx.x;
    cp[threadIdx.x] = (sl < ns && slots[sl].pm_copy) ? 1 : 0;
    if (cp[threadIdx.x]) any = 1;
  }
  __syncthreads();
  if (!any) return;
  const int c = threadIdx.x % FT, r0 = threadIdx.x / FT;
  for (int64_t i0 = (int64_t)blockIdx.x * FT; i0 < n; i0 += (int64_t)gridDim.x * FT) {
    for (int r = r0; r < FT; r += NT / FT) {
      const int64_t i = i0 + r;
      const int sl = s0 + c;
      t[r][c] = (i < n && sl < nqp) ? D[i * nqp + sl] : 0u;
    }
    __syncthreads();
    for (int r = r0; r < FT; r += NT / FT) {
      const int sl = s0 + r;
      const int64_t i = i0 + c;
      if (sl < ns && i < n && cp[r]) B.S[(int64_t)sl * n + i] = (int64_t)t[c][r];
    }
    __syncthreads();
  }
}

template <int DT>
__device__ void finalize(Slot *sl, int s, const QDesc &qd, const uint8_t *X, const Bufs &B,
                         const Geometry &G) {
  const int64_t n = G.n, m = G.m;
  const SlotArrays a = slot_arrays(B, n, s, sl->par);
  const int kh = sl->kh;
  __shared__ SelScratch ss;
  __shared__ uint64_t skey[kMaxKH];
  __shared__ int32_t sidx[kMaxKH];
  __shared__ int cnt;
  __shared__ int64_t red[MT / kWave];
  const int n_act = sl->n_act, n_xa = sl->n_xa, n_acc = sl->n_acc;
  const int64_t nP = (int64_t)n_act + n_xa + n_acc;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  if (nP > kh) {
    const uint8_t *q = reinterpret_cast<const uint8_t *>(sl->q);
    int64_t made = 0, cost = 0;
    for (int t = 0; t < n_acc; ++t) {
      const int32_t i = a.acc[t];
      if (a.fl[i] & FL_EXACT) continue;
      cost += sl->norepl ? m - (int64_t)sl->T[a.ri[i]] : m;
      const int64_t tot = block_exact_sum<DT, MT>(X, m, i, q, sl->F, G.metric, red);
      if (threadIdx.x == 0) {
        a.S[i] = tot;
        a.fl[i] = a.fl[i] | FL_EXACT;
      }
      ++made;
      __syncthreads();
    }
    if (threadIdx.x == 0 && made) {
      sl->exact_points += made;
      sl->coord_evals += cost;
    }
    __syncthreads();
    // P = [xa | acc] (n_act == 0 here), every point exact
    const double denom = (double)m * sl->W;
    auto elem = [&](int64_t p) -> int32_t { return p < n_xa ? a.xa[p] : a.acc[p - n_xa]; };
    auto gk = [&](int64_t p) -> uint64_t { return dkey((double)a.S[elem(p)] / denom); };
    const int64_t N = (int64_t)n_xa + n_acc;
    int less;
    const uint64_t v = block_kth_gen<MT>(N, gk, kh, ss, &less);
    const uint32_t thr = block_kth_u32_gen<MT>(
        N, [&](int64_t p) { return (uint32_t)elem(p); }, [&](int64_t p) { return gk(p) == v; },
        kh - less, ss);
    for (int64_t p = threadIdx.x; p < N; p += MT) {
      const int32_t i = elem(p);
      const uint64_t kk = gk(p);
      if (kk < v || (kk == v && (uint32_t)i <= thr)) {
        const int pos = atomicAdd(&cnt, 1);
        if (pos < kMaxKH) {
          skey[pos] = kk;
          sidx[pos] = i;
        }
      }
    }
  } else {
    for (int64_t p = threadIdx.x; p < nP; p += MT) {
      const int32_t i = elem_P(sl, a, p);
      double d, al;
      point_bounds(sl, m, a.S[i], a.fl[i], a.ri[i], d, al);
      skey[p] = dkey(d);
      sidx[p] = i;
    }
    if (threadIdx.x == 0) cnt = (int)nP;
  }
  __syncthreads();
  const int c = min(cnt, kh);
  int len = 1;
  while (len < c) len <<= 1;
  for (int p = c + (int)threadIdx.x; p < len; p += MT) {
    skey[p] = ~0ull;
    sidx[p] = 0x7FFFFFFF;
  }
  block_bitonic_sort<MT>(skey, sidx, len);
  for (int64_t j = threadIdx.x; j < qd.out_stride; j += MT) qd.out_idx[j] = j < c ? (int64_t)sidx[j] : -1;
  if (threadIdx.x == 0) {
    *qd.out_count = c;
    if (qd.out_stats) {
      qd.out_stats->coord_evals = sl->coord_evals;
      qd.out_stats->rounds = sl->rounds;
      qd.out_stats->count = c;
      qd.out_stats->exact_points = sl->exact_points;
    }
  }
  __syncthreads();
}

// Claims at most one query for an idle slot and initialises it.  A trivial
// query (k+h >= n, or a zero value range) is answered on the spot and the
// slot stays idle until the next step.  There is deliberately no loop here:
// a loop whose head and back-edge both hold thread-0-only work around
// barriers can be restructured so that lane 0 leaves the loop nest while the
// rest of its wave keeps iterating.
// direct: slot s takes query s (s < nq) without touching the shared counter,
// which the host has already set past those queries (first admission of a
// batch: one compare-and-swap per slot on one counter would serialise them).
__device__ void admit(Slot *sl, const QDesc *qd, const Sched *sched, Ctl *ctl, int64_t n, int64_t m,
                      bool direct) {
  __shared__ int claimed;
  if (direct) {
    if (threadIdx.x == 0) claimed = (int)blockIdx.x < ctl->nq ? (int)blockIdx.x : -1;
  } else if (threadIdx.x == 0) {
    const int nq = __atomic_load_n(&ctl->nq, __ATOMIC_RELAXED);
    int cur = __atomic_load_n(&ctl->next_query, __ATOMIC_RELAXED);
    int got = -1;
    while (cur < nq) {
      const int prev = atomicCAS(&ctl->next_query, cur, cur + 1);
      if (prev == cur) {
        got = cur;
        break;
      }
      cur = prev;
    }
    claimed = got;
  }
  __syncthreads();
  const int qseq = claimed;
  if (qseq < 0) return;
  const int qi = ctl->qcap > 0 ? qseq % ctl->qcap : qseq;  // ring slot of the query
  const QDesc &d = qd[qi];
  if (d.trivial) {
    write_trivial(d, n);
    if (threadIdx.x == 0) {
      __threadfence();
      atomicAdd(&ctl->done, 1);
    }
    return;
  }
  const Sched &sc = sched[d.sched];
  for (int r = threadIdx.x; r < kMaxRounds; r += blockDim.x) {
    sl->T[r] = sc.T[r];
    sl->alpha[r] = sc.alpha[r];
  }
  if (threadIdx.x == 0) {
    sl->qi = qi;
    sl->cur = 0;
    sl->par = 0;
    sl->implicit = 1;
    sl->n_act = (int32_t)n;
    sl->n_xa = 0;
    sl->n_acc = 0;
    sl->nn_act = 0;
    sl->nn_xa = 0;
    sl->nn_acc = 0;
    sl->k = d.k;
    sl->kh = d.kh;
    sl->R = sc.R;
    sl->c_exact = d.c_exact;
    sl->F = d.F;
    sl->norepl = d.norepl;
    sl->shared = d.shared;
    sl->seed = d.seed;
    sl->W = d.W;
    sl->q = d.q;
    sl->rounds = 0;
    sl->pm_copy = 0;
    sl->coord_evals = sc.R == 0 ? n * m : n * (int64_t)sc.T[0];
    sl->exact_points = sc.R == 0 ? n : 0;
    sl->state = 1;
  }
}

template <int DT>
__global__ __launch_bounds__(MT) void k_finish(Slot *__restrict__ slots, const QDesc *__restrict__ qd,
                                               const Sched *__restrict__ sched, Ctl *ctl,
                                               const uint8_t *__restrict__ X, Bufs B, Geometry G,
                                               int admit_only) {
  const int s = blockIdx.x;
  Slot *sl = &slots[s];
  const int64_t n = G.n, m = G.m;
  if (sl->state == 1 && !admit_only) {
    const bool dense = G.flagsets && sl->implicit != 0;  // (uniform over the block)
    if (threadIdx.x == 0) sl->pm_copy = 0;  // (copied after the previous step's k_finish)
    if (dense) {
      // this round's counts, one record per point tile of k_decide_pm
      const int64_t nt = (n + DQ_PT - 1) / DQ_PT;
      const uint32_t *rec = reinterpret_cast<const uint32_t *>(B.part + (int64_t)s * B.part_stride);
      int64_t c3[3] = {0, 0, 0};
      for (int64_t t = threadIdx.x; t < nt; t += MT)
        for (int k = 0; k < 3; ++k) c3[k] += rec[3 * t + k];
      __shared__ int64_t red3[MT / kWave][3];
      for (int k = 0; k < 3; ++k)
        for (int o = kWave / 2; o > 0; o >>= 1) c3[k] += shfl_xor_i64(c3[k], o);
      if (lane_id() == 0)
        for (int k = 0; k < 3; ++k) red3[threadIdx.x / kWave][k] = c3[k];
      __syncthreads();
      if (threadIdx.x == 0) {
        int64_t t3[3] = {0, 0, 0};
        for (int w = 0; w < MT / kWave; ++w)
          for (int k = 0; k < 3; ++k) t3[k] += red3[w][k];
        sl->nn_act = (int32_t)t3[0];
        sl->nn_xa = (int32_t)t3[1];
        sl->nn_acc = sl->n_acc + (int32_t)t3[2];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      sl->n_act = sl->nn_act;
      sl->n_xa = sl->nn_xa;
      sl->n_acc = sl->nn_acc;
      sl->rounds += 1;
      sl->implicit = dense ? 2 : 0;
      sl->par ^= 1;
    }
    __syncthreads();
    const int64_t nP = (int64_t)sl->n_act + sl->n_xa + sl->n_acc;
    if (ctl->stop_after > 0 && sl->rounds >= ctl->stop_after) {
      if (dense) {  // the slot-major state of the inspected slot, from the point-major sums
        const SlotArrays a = slot_arrays(B, n, s, sl->par);
        for (int64_t i = threadIdx.x; i < n; i += MT) {
          a.S[i] = (int64_t)B.dpm[i * B.dpm_stride + s];
          if (a.fl[i] == 0) a.ri[i] = (uint8_t)sl->cur;
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        sl->state = 2;  // frozen for inspection
        atomicAdd(&ctl->done, 1);
      }
      return;
    }
    if (nP <= sl->kh || sl->n_act == 0) {
      if (sl->implicit == 2) lists_from_flags(sl, s, B, G);
      finalize<DT>(sl, s, qd[sl->qi], X, B, G);
      if (threadIdx.x == 0) {
        sl->state = 0;
        atomicAdd(&ctl->done, 1);
      }
      __syncthreads();
    } else {
      // a dense slot of a point-major batch whose undecided set has become
      // small continues in list form (per-slot kernels cost per undecided
      // point, the point-major ones per point of the DB)
      if (sl->implicit == 2 && G.sparse_div > 0 && ((int64_t)sl->n_act + sl->n_xa) * G.sparse_div <= n)
        lists_from_flags(sl, s, B, G, true);
      if (threadIdx.x == 0) {
        const int cur = sl->cur + 1;
        sl->cur = cur;
        // the exact round costs m per point, or the m - T not yet seen without replacement
        const int64_t per = cur < sl->R ? (int64_t)(sl->T[cur] - sl->T[cur - 1])
                                        : (sl->norepl ? m - (int64_t)sl->T[cur - 1] : m);
        sl->coord_evals += per * sl->n_act;
        if (cur >= sl->R) sl->exact_points += sl->n_act;
        sl->nn_act = 0;
        sl->nn_xa = 0;
        sl->nn_acc = sl->n_acc;
      }
      return;
    }
  }
  if (sl->state == 0 && !G.packed_admit) admit(sl, qd, sched, ctl, n, m, admit_only == 2);
}

// Packed admission (one block): the queries submitted but not yet admitted
// go to the lowest idle slots, in slot order, so that running slots stay
// packed at the bottom of the engine; then Ctl::run_hi = 1 + the highest
// running slot, which bounds the slots the next step's kernels cover.
__global__ __launch_bounds__(MT) void k_admit_packed(Slot *__restrict__ slots, const QDesc *__restrict__ qd,
                                                     const Sched *__restrict__ sched, Ctl *ctl, int64_t n,
                                                     int64_t m, int32_t ns) {
  __shared__ int base, wsum[MT / kWave], hi;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  if (threadIdx.x == 0) {
    base = 0;
    hi = 0;
  }
  __syncthreads();
  const int nq = ctl->nq, first = ctl->next_query;
  for (int s0 = 0; s0 < ns; s0 += MT) {
    const int s = s0 + (int)threadIdx.x;
    const bool idle = s < ns && slots[s].state == 0;
    // rank of this idle slot among the idle slots below it
    const uint64_t bal = __ballot(idle);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    int before = base;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    const int rank = before + __popcll(bal & lt);
    const int qseq = first + rank;
    if (idle && qseq < nq) {
      Slot *sl = &slots[s];
      const int qi = ctl->qcap > 0 ? qseq % ctl->qcap : qseq;
      const QDesc &d = qd[qi];
      if (d.trivial) {
        const int64_t cnt = d.kh < n ? d.kh : n;
        for (int64_t j = 0; j < d.out_stride; ++j) d.out_idx[j] = j < cnt ? j : -1;
        *d.out_count = (int32_t)cnt;
        if (d.out_stats) {
          d.out_stats->coord_evals = 0;
          d.out_stats->rounds = 0;
          d.out_stats->count = (int32_t)cnt;
          d.out_stats->exact_points = 0;
        }
        __threadfence();
        atomicAdd(&ctl->done, 1);
      } else {
        const Sched &sc = sched[d.sched];
        for (int r = 0; r < kMaxRounds; ++r) {
          sl->T[r] = sc.T[r];
          sl->alpha[r] = sc.alpha[r];
        }
        sl->qi = qi;
        sl->cur = 0;
        sl->par = 0;
        sl->implicit = 1;
        sl->n_act = (int32_t)n;
        sl->n_xa = 0;
        sl->n_acc = 0;
        sl->nn_act = 0;
        sl->nn_xa = 0;
        sl->nn_acc = 0;
        sl->k = d.k;
        sl->kh = d.kh;
        sl->R = sc.R;
        sl->c_exact = d.c_exact;
        sl->F = d.F;
        sl->norepl = d.norepl;
        sl->shared = d.shared;
        sl->seed = d.seed;
        sl->W = d.W;
        sl->q = d.q;
        sl->rounds = 0;
        sl->pm_copy = 0;
        sl->coord_evals = sc.R == 0 ? n * m : n * (int64_t)sc.T[0];
        sl->exact_points = sc.R == 0 ? n : 0;
        sl->state = 1;
      }
    }
    if (s < ns && slots[s].state == 1) atomicMax(&hi, s + 1);
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < MT / kWave; ++w) tot += wsum[w];
      base += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int took = min(base, max(0, nq - first));
    ctl->next_query = first + took;
    ctl->run_hi = hi;
  }
}

// ---------------------------------------------------------------- launch table

}  // namespace knn

// Host-side launchers (called from the runtime).
namespace knn {

// max_list: the longest list expected (the grid covers it in one pass; the
// kernel's chunk loop covers longer ones)
template <int DT, int MET>
static void launch_sample_dt(Slot *slots, const uint8_t *X, const Bufs &B, const Geometry &G, bool qlds,
                             size_t qbytes, hipStream_t st, int64_t max_list) {
  dim3 grid((unsigned)G.nslots, (unsigned)std::max<int64_t>(1, (max_list + G.ch_sample - 1) / G.ch_sample));
  if (qlds)
    hipLaunchKernelGGL((k_sample<DT, MET, true>), grid, dim3(NT), qbytes, st, slots, X, B, G);
  else
    hipLaunchKernelGGL((k_sample<DT, MET, false>), grid, dim3(NT), 0, st, slots, X, B, G);
}

template <int DT>
static void launch_sample_met(Slot *slots, const uint8_t *X, const Bufs &B, const Geometry &G, bool qlds,
                              size_t qbytes, hipStream_t st, int64_t max_list = -1) {
  if (max_list < 0) max_list = G.n;
  if (G.metric == KNN_METRIC_L1)
    launch_sample_dt<DT, KNN_METRIC_L1>(slots, X, B, G, qlds, qbytes, st, max_list);
  else
    launch_sample_dt<DT, KNN_METRIC_L2>(slots, X, B, G, qlds, qbytes, st, max_list);
}

void launch_prep_f32(QDesc *qd, int32_t nq, int64_t n, int64_t m, double lo, double hi, int32_t metric,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_prep_f32, dim3((unsigned)nq), dim3(NT), 0, st, qd, nq, n, m, lo, hi, metric);
}

// the exact round of query-lane batches (k_naive.hip: shares the scan's GEMM tile)
void launch_exact_ql_u8(const Slot *slots, const int8_t *Q8, const int32_t *qn, const int8_t *X8, const int32_t *xn,
                        const Bufs &B, const Geometry &G, int32_t cur, int32_t impl, uint32_t *Dpm, int32_t nqp,
                        hipStream_t st);

// rounds of a batch that shares one coordinate sequence (k_naive.hip: the same tiles)
void launch_round_seq_u8(const Slot *slots, const SeqBufs &q, int32_t lo, int32_t hi, int64_t t0, int64_t t1,
                         const uint8_t *A, uint32_t *D, int32_t nqp, const Bufs &B, const Geometry &G, int32_t cur,
                         int32_t impl, int32_t exact, hipStream_t st);

int stage_rows_for(int64_t m, int64_t mp, int want) {
  // LDS: the transposed query tile (GRP x mp) plus the row tile (rows x m)
  constexpr int64_t kLds = 160 * 1024 - 4096;  // static shared memory of the kernel stays below 4 KB
  int rows = 64;
  while (rows > want || (rows >= 8 && GRP * mp + rows * m > kLds)) rows >>= 1;
  return rows >= 8 ? rows : 0;
}

void launch_build_qt(const Slot *slots, int32_t ns, int64_t m, int32_t nqp, uint8_t *qt, hipStream_t st) {
  const int64_t total = m * (int64_t)nqp;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + NT - 1) / NT, 4096);
  hipLaunchKernelGGL(k_build_qt, dim3(blocks), dim3(NT), 0, st, slots, ns, m, nqp, qt);
}

constexpr size_t kSeqGatherLds = 160 * 1024 - 4096;  // dynamic LDS a gather block may take

void launch_seq_prepare_f32(const Slot *slots, int32_t ns, const float *X, int64_t n, int64_t m, uint64_t seed,
                            int32_t norepl, const SeqBufs &q, hipStream_t st) {
  const unsigned cb = (unsigned)std::min<int64_t>((q.kp / 4 + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(k_seq_coords, dim3(cb), dim3(NT), 0, st, seed, norepl, m, q.tlen, q.kp, q.js);
  const size_t lds = (size_t)m * 4;
  const unsigned gx = (unsigned)std::min<int64_t>(n, 8192), gq = (unsigned)std::max<int32_t>(1, ns);
  if (lds <= 65536) {
    hipLaunchKernelGGL((k_seq_gather_f32<false, true>), dim3(gx), dim3(NT), lds, st, X, slots, n, m, q.js, q.kp,
                       q.xf);
    hipLaunchKernelGGL((k_seq_gather_f32<true, true>), dim3(gq), dim3(NT), lds, st, X, slots, (int64_t)ns, m, q.js,
                       q.kp, q.qf);
  } else {
    hipLaunchKernelGGL((k_seq_gather_f32<false, false>), dim3(gx), dim3(NT), 0, st, X, slots, n, m, q.js, q.kp,
                       q.xf);
    hipLaunchKernelGGL((k_seq_gather_f32<true, false>), dim3(gq), dim3(NT), 0, st, X, slots, (int64_t)ns, m, q.js,
                       q.kp, q.qf);
  }
}

// Whether any slot is running (dense: and holds its sets as flags; the exact
// round's product over the gathered copies runs only for those).
__global__ __launch_bounds__(1024) void k_seq_any_dense(const Slot *__restrict__ slots, int32_t ns,
                                                        int32_t *__restrict__ flag, int32_t dense) {
  bool any = false;
  for (int s = threadIdx.x; s < ns; s += 1024)
    any = any || (slots[s].state == 1 && (!dense || slots[s].implicit != 0));
  const int r = __syncthreads_or(any ? 1 : 0);
  if (threadIdx.x == 0) *flag = r ? 1 : 0;
}

// The gather of the point rows (or, QUERIES, the slots' query rows) over
// columns [c0, c1), or nothing when need is set and reads 0 at run time.
// Staged rows take m + 16 bytes of LDS and the coordinates of a launch two bytes
// each: a column range whose coordinates do not fit beside the row is split
// into launches of whole 64-column pieces (each stages the rows again).
template <bool QUERIES>
static void launch_seq_gather_cols(const Slot *slots, int32_t ns, const uint8_t *X, int64_t rows, int64_t m,
                                   int32_t metric, const SeqBufs &q, int8_t *out, int64_t c0, int64_t c1,
                                   const int32_t *need, hipStream_t st) {
  const unsigned grid = (unsigned)(QUERIES ? rows : std::min<int64_t>(rows, 8192));
  const int64_t mr = (m + 15) / 16 * 16;
  const int64_t room = ((int64_t)kSeqGatherLds - mr - 16) / 2 / 64 * 64;  // coordinates per staged launch
  const bool stage = m < 65536 && room >= 64;
  const int64_t step = stage ? room : (c1 - c0);
  for (int64_t a = c0; a < c1; a += step) {
    const int64_t b = std::min(c1, a + step);
    const size_t lds = (size_t)(mr + 16 + 2 * (b - a));
#define KNN_SEQ_GATHER_LAUNCH(MET_)                                                                                \
  do {                                                                                                             \
    if (stage && lds > 40 * 1024) {                                                                                \
      if (lds > 65536)                                                                                             \
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_seq_gather<MET_, QUERIES, true, 1024>),         \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSeqGatherLds);                \
      hipLaunchKernelGGL((k_seq_gather<MET_, QUERIES, true, 1024>), dim3(grid), dim3(1024), lds, st, X, slots, ns, \
                         rows, m, q.js, q.kp, out, a, b, need);                                                    \
    } else if (stage) {                                                                                            \
      hipLaunchKernelGGL((k_seq_gather<MET_, QUERIES, true>), dim3(grid), dim3(NT), lds, st, X, slots, ns, rows,  \
                         m, q.js, q.kp, out, a, b, need);                                                          \
    } else {                                                                                                       \
      hipLaunchKernelGGL((k_seq_gather<MET_, QUERIES, false>), dim3(grid), dim3(NT), 0, st, X, slots, ns, rows, m, \
                         q.js, q.kp, out, a, b, need);                                                             \
    }                                                                                                              \
  } while (0)
    if (metric == KNN_METRIC_L1)
      KNN_SEQ_GATHER_LAUNCH(KNN_METRIC_L1);
    else
      KNN_SEQ_GATHER_LAUNCH(KNN_METRIC_L2);
#undef KNN_SEQ_GATHER_LAUNCH
  }
}

void launch_seq_prepare(const Slot *slots, const Sched *sc, int32_t ns, int32_t nqp, const uint8_t *X, int64_t n,
                        int64_t m, uint64_t seed, int32_t norepl, int32_t metric, const SeqBufs &q,
                        const int32_t *xnorm, const int32_t *qnorm, int64_t ca, int32_t ba, hipStream_t st) {
  const unsigned cb = (unsigned)std::min<int64_t>((q.kp / 4 + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(k_seq_coords, dim3(cb), dim3(NT), 0, st, seed, norepl, m, q.tlen, q.kp, q.js);
  const unsigned gx = (unsigned)std::min<int64_t>(n, 8192), gq = (unsigned)nqp;
  // the queries' rows at every column (they are few), with all their norms;
  // the points' rows at the first rounds' columns [0, ca), with the norms at
  // the boundaries below ba (the later columns: launch_seq_gather_more)
  launch_seq_gather_cols<false>(slots, ns, X, n, m, metric, q, q.xs, 0, ca, nullptr, st);
  launch_seq_gather_cols<true>(slots, ns, X, (int64_t)nqp, m, metric, q, q.qs, 0, q.kp, nullptr, st);
  if (metric == KNN_METRIC_L2) {
    hipLaunchKernelGGL(k_seq_norms, dim3(gx), dim3(NT), 0, st, q.xs, n, q.kp, sc, q.nb, m, xnorm, q.xn, n, 0, ba,
                       (const int32_t *)nullptr);
    hipLaunchKernelGGL(k_seq_norms, dim3(gq), dim3(NT), 0, st, q.qs, (int64_t)nqp, q.kp, sc, q.nb, m, qnorm, q.qn,
                       (int64_t)nqp, 0, q.nb, (const int32_t *)nullptr);
  }
}

void launch_seq_gather_more(const Slot *slots, int32_t ns, const Sched *sc, const uint8_t *X, int64_t n, int64_t m,
                            int32_t metric, const SeqBufs &q, int64_t c0, int64_t c1, int32_t b0, int32_t b1,
                            int32_t dense, const int32_t *xnorm, hipStream_t st) {
  if (c0 >= c1 && b0 >= b1) return;
  int32_t *flag = q.flag + (dense ? 1 : 0);
  hipLaunchKernelGGL(k_seq_any_dense, dim3(1), dim3(1024), 0, st, slots, ns, flag, dense);
  if (c0 < c1) launch_seq_gather_cols<false>(slots, ns, X, n, m, metric, q, q.xs, c0, c1, flag, st);
  if (metric == KNN_METRIC_L2 && b0 < b1) {
    const unsigned gx = (unsigned)std::min<int64_t>(n, 8192);
    hipLaunchKernelGGL(k_seq_norms, dim3(gx), dim3(NT), 0, st, q.xs, n, q.kp, sc, q.nb, m, xnorm, q.xn, n, b0, b1,
                       (const int32_t *)flag);
  }
}

// Point blocks of a query-lane sampling launch (each walks a contiguous
// range of points).  KNN_QL_BLOCKS overrides the default.
static unsigned ql_blocks_x(int64_t n) {
  const char *e = std::getenv("KNN_QL_BLOCKS");
  const int64_t want = e ? std::max<int64_t>(1, std::atoll(e)) : 2048;
  return (unsigned)std::min<int64_t>((n + QL_NW - 1) / QL_NW, want);
}

// Points of a slot's list that the per-slot grids of a point-major batch
// cover in one pass: a slot there turns sparse with at most n / sparse_div
// undecided points (plus its accepted ones); longer lists take more passes
// of the kernels' chunk loops.  KNN_SPARSE_LIST overrides it.
static int64_t sparse_list_len(const Geometry &G) {
  if (const char *e = std::getenv("KNN_SPARSE_LIST")) return std::max<int64_t>(1, std::atoll(e));
  return G.sparse_div > 0 ? std::min<int64_t>(G.n, G.n / G.sparse_div + kWave) : 1;
}

void launch_step(Slot *slots, const QDesc *qd, const Sched *sched, Ctl *ctl, const uint8_t *X,
                 const Bufs &B, const Geometry &G0, bool any_cexact, hipStream_t st, int sample_kind,
                 int stage_rows, const QlRound *ql, const uint8_t *qt, int32_t nqp, uint32_t *qd_buf,
                 const int8_t *q8, const int32_t *q8n, const SeqBufs *seq) {
  Geometry G = G0;
  G.prof = prof_device_counters();
  G.stage = (G.dtype == KNN_U8 && G.grouped) ? stage_rows : 0;
  const int elem = G.dtype == KNN_U8 ? 1 : 4;
  const size_t qbytes = (size_t)G.m * elem;
  const bool qlds = qbytes <= 48 * 1024;
  const unsigned ns = (unsigned)G.nslots;
  if (G.flagsets && ql && qt && qd_buf && q8 && q8n && G.dtype == KNN_U8) {
    // A query-lane batch that keeps its sums point-major: sampling (or the
    // exact round) accumulates into D, then selection and decisions read D
    // in tiles; no slot-major sums, no lists, no transposes.
    uint8_t *A = reinterpret_cast<uint8_t *>(qd_buf + G.n * (int64_t)nqp);  // follows D in the arena
    if (seq && seq->xs && (!ql->exact || ql->norepl)) {
      // one coordinate sequence for all points: the round's columns of the
      // gathered copies, as one product over (queries x points)
      const int tk = prof_begin(ql->exact ? PROF_EXACT : PROF_SAMPLE, st);
      launch_round_seq_u8(slots, *seq, ql->cur, ql->cur + 1, ql->t0, ql->t1, A, qd_buf, nqp, B, G, ql->cur, ql->impl,
                          ql->exact, st);
      prof_end(tk, st, 0.0);
    } else if (ql->exact) {
      const int tk = prof_begin(PROF_EXACT, st);
      launch_exact_ql_u8(slots, q8, q8n, G.x8, G.xn, B, G, ql->cur, ql->impl, qd_buf, nqp, st);
      prof_end(tk, st, 0.0);
    } else {
      const unsigned bx = ql_blocks_x(G.n);
      const unsigned by = (unsigned)((nqp + QL_SLOTS - 1) / QL_SLOTS);
      const int tk = prof_begin(PROF_SAMPLE, st);
      if (G.metric == KNN_METRIC_L1)
        hipLaunchKernelGGL(k_sample_ql_u8<KNN_METRIC_L1>, dim3(bx, by), dim3(QL_BT), 0, st, slots, X, qt, nqp, A,
                           qd_buf, B, G, *ql);
      else
        hipLaunchKernelGGL(k_sample_ql_u8<KNN_METRIC_L2>, dim3(bx, by), dim3(QL_BT), 0, st, slots, X, qt, nqp, A,
                           qd_buf, B, G, *ql);
      prof_end(tk, st, 0.0);
    }
    // slots that turned sparse: per-slot sampling over their lists (or their
    // exact sums in the exact round); the kernel skips the dense slots
    const int64_t sparse_list = sparse_list_len(G);
    int tk = prof_begin(PROF_SPARSE, st);
    if (seq && seq->xs && !ql->exact) {
      // shared sequence: the sparse slots' samples are columns of the gathered rows
      // (a few blocks per slot, looping over the list: with no sparse slot
      // the launch is 16 blocks per slot that leave at once)
      const dim3 grid(ns, (unsigned)std::max<int64_t>(1, std::min<int64_t>((sparse_list + SEQ_SP - 1) / SEQ_SP, 16)));
      if (G.metric == KNN_METRIC_L1)
        hipLaunchKernelGGL(k_sample_seq_sparse<KNN_METRIC_L1>, grid, dim3(NT), 0, st, slots, *seq, B, G);
      else
        hipLaunchKernelGGL(k_sample_seq_sparse<KNN_METRIC_L2>, grid, dim3(NT), 0, st, slots, *seq, B, G);
    } else {
      launch_sample_met<KNN_U8>(slots, X, B, G, qlds, qbytes, st, sparse_list);
    }
    prof_end(tk, st, 0.0);
    tk = prof_begin(PROF_SELECT, st);
    const int64_t nsel = ((G.n + FS_PT - 1) / FS_PT) * ((nqp + FS_SL - 1) / FS_SL);
    if (G.kmax + 1 > kWave)
      hipLaunchKernelGGL(k_select_pm<true>, dim3((unsigned)xcd_grid(nsel)), dim3(FS_NT), 0, st, slots, qd_buf, nqp, B, G,
                         ql->cur, (ql->cur == 0 && !ql->exact) ? 1 : 0);
    else
      hipLaunchKernelGGL(k_select_pm<false>, dim3((unsigned)xcd_grid(nsel)), dim3(FS_NT), 0, st, slots, qd_buf, nqp, B, G,
                         ql->cur, (ql->cur == 0 && !ql->exact) ? 1 : 0);
    hipLaunchKernelGGL(k_select_pm_mixed, dim3(ns), dim3(kWave), 0, st, slots, qd_buf, nqp, B, G, ql->cur,
                       (ql->cur == 0 && !ql->exact) ? 1 : 0);
    hipLaunchKernelGGL(k_select_partial, dim3((unsigned)((sparse_list + SEL_CH - 1) / SEL_CH), ns), dim3(NT), 0, st,
                       slots, B, G);
    hipLaunchKernelGGL(k_select_merge_pm, dim3(ns), dim3(SMP_T), 0, st, slots, B, G);
    hipLaunchKernelGGL(k_select_merge, dim3(ns), dim3(MT), 0, st, slots, B, G, 1);
    prof_end(tk, st, 0.0);
    tk = prof_begin(PROF_DECIDE, st);
    const int64_t ndec = ((G.n + DQ_PT - 1) / DQ_PT) * ((nqp + DQ_SL - 1) / DQ_SL);
    hipLaunchKernelGGL(k_decide_pm, dim3((unsigned)xcd_grid(ndec)), dim3(NT), 0, st, slots, qd_buf, A, nqp, B, G,
                       ql->cur);
    hipLaunchKernelGGL(k_decide, dim3((unsigned)((sparse_list + DEC_CH - 1) / DEC_CH), ns), dim3(NT), 0, st, slots,
                       B, G);
    prof_end(tk, st, 0.0);
    tk = prof_begin(PROF_FINISH, st);
    if (G.dtype == KNN_U8)
      hipLaunchKernelGGL(k_finish<KNN_U8>, dim3(ns), dim3(MT), 0, st, slots, qd, sched, ctl, X, B, G, 0);
    // slots that turned sparse in this step: their sums, slot-major
    const dim3 ct((unsigned)std::min<int64_t>((G.n + FT - 1) / FT, 128), (unsigned)((nqp + FT - 1) / FT));
    hipLaunchKernelGGL(k_pm_to_slot, ct, dim3(NT), 0, st, slots, qd_buf, nqp, B, G);
    prof_end(tk, st, 0.0);
    return;
  }
  // exact round of a query-lane batch: one GEMM over (slots x points)
  const bool ql_exact = ql && ql->exact && q8 && q8n && G.dtype == KNN_U8;
  if (ql_exact) {
    const int tk = prof_begin(PROF_EXACT, st);
    launch_exact_ql_u8(slots, q8, q8n, G.x8, G.xn, B, G, ql->cur, ql->impl, qd_buf, nqp, st);
    prof_end(tk, st, 0.0);
    ql = nullptr;  // the rest of the step as usual
  }
  const bool use_ql = ql && !ql->exact && qt && qd_buf && G.dtype == KNN_U8;
  int tok = (use_ql || ql_exact) ? -1 : prof_begin(sample_kind == 1 ? PROF_EXACT : PROF_SAMPLE, st);
  if (ql_exact) {
    // sampling done above
  } else if (use_ql) {
    const unsigned bx = ql_blocks_x(G.n);
    const unsigned by = (unsigned)((nqp + QL_SLOTS - 1) / QL_SLOTS);
    uint8_t *A = reinterpret_cast<uint8_t *>(qd_buf + G.n * (int64_t)nqp);  // follows D in the arena
    const dim3 tiles((unsigned)((G.n + FT - 1) / FT), (unsigned)((nqp + FT - 1) / FT));
    if (!ql->impl) {
      tok = prof_begin(PROF_QL_AUX, st);
      hipLaunchKernelGGL(k_flags_ql, tiles, dim3(NT), 0, st, slots, A, nqp, B, G, ql->cur);
      prof_end(tok, st, 0.0);
    }
    tok = prof_begin(PROF_SAMPLE, st);
    if (G.metric == KNN_METRIC_L1)
      hipLaunchKernelGGL(k_sample_ql_u8<KNN_METRIC_L1>, dim3(bx, by), dim3(QL_BT), 0, st, slots, X, qt, nqp, A, qd_buf,
                         B, G, *ql);
    else
      hipLaunchKernelGGL(k_sample_ql_u8<KNN_METRIC_L2>, dim3(bx, by), dim3(QL_BT), 0, st, slots, X, qt, nqp, A, qd_buf,
                         B, G, *ql);
    prof_end(tok, st, 0.0);
    tok = prof_begin(PROF_QL_AUX, st);
    hipLaunchKernelGGL(k_fold_ql, tiles, dim3(NT), 0, st, slots, qd_buf, nqp, B, G, ql->cur);
  } else if (G.dtype == KNN_U8 && G.grouped) {
    size_t gbytes = std::max<size_t>((size_t)GRP * G.mp + 8 * GRP, qbytes);
    if (G.stage > 0) {
      gbytes = std::max<size_t>(gbytes, (size_t)GRP * G.mp + (size_t)G.stage * G.m);
      static bool attr_set = false;
      if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_sample_grp_u8<KNN_METRIC_L2>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_sample_grp_u8<KNN_METRIC_L1>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
        attr_set = true;
      }
    }
    dim3 grid((unsigned)((G.nslots + GRP - 1) / GRP), (unsigned)((G.n + G.ch_sample - 1) / G.ch_sample));
    if (G.metric == KNN_METRIC_L1)
      hipLaunchKernelGGL(k_sample_grp_u8<KNN_METRIC_L1>, grid, dim3(GBT), gbytes, st, slots, X, G.x8, G.xn, G.mp, B, G);
    else
      hipLaunchKernelGGL(k_sample_grp_u8<KNN_METRIC_L2>, grid, dim3(GBT), gbytes, st, slots, X, G.x8, G.xn, G.mp, B, G);
  } else if (G.dtype == KNN_U8) {
    launch_sample_met<KNN_U8>(slots, X, B, G, qlds, qbytes, st);
  } else if (sample_kind == 1 || (seq && seq->xf && ql && (!ql->exact || ql->norepl))) {
    // a lock-step fp32 batch (every running slot is at this round): its exact
    // round as one tiled pass over (slots x points); with a shared coordinate
    // sequence also its sampled rounds (columns of the gathered copies), and
    // without replacement the exact round adds the columns not yet sampled
    const int64_t nwork = ((G.nslots + XF_Q - 1) / XF_Q) * ((G.n + XF_P - 1) / XF_P);
    const bool on_seq = seq && seq->xf && ql && (!ql->exact || ql->norepl);
    const float *Xf = on_seq ? seq->xf : reinterpret_cast<const float *>(X);
    const int64_t stride = on_seq ? seq->kp : G.m;
    const int64_t c0 = on_seq ? (int64_t)ql->t0 : 0, c1 = on_seq ? (int64_t)ql->t1 : G.m;
    const int32_t mode = !on_seq ? 0 : (ql->exact ? 2 : 1);
    const int32_t cur = ql ? ql->cur : -1;
    const float *QS = on_seq ? seq->qf : nullptr;
    if (G.metric == KNN_METRIC_L1)
      hipLaunchKernelGGL(k_exact_f32_tile<KNN_METRIC_L1>, dim3((unsigned)xcd_grid(nwork)), dim3(NT), 0, st, slots, Xf,
                         stride, c0, c1, QS, mode, cur, B, G);
    else
      hipLaunchKernelGGL(k_exact_f32_tile<KNN_METRIC_L2>, dim3((unsigned)xcd_grid(nwork)), dim3(NT), 0, st, slots, Xf,
                         stride, c0, c1, QS, mode, cur, B, G);
  } else {
    launch_sample_met<KNN_F32>(slots, X, B, G, qlds, qbytes, st);
  }
  prof_end(tok, st, 0.0);
  if (any_cexact) {
    tok = prof_begin(PROF_CAND, st);
    hipLaunchKernelGGL(k_cand_partial, dim3((unsigned)((G.n + CAND_CH - 1) / CAND_CH), ns), dim3(NT), 0, st,
                       slots, B, G);
    if (G.dtype == KNN_U8)
      hipLaunchKernelGGL(k_cand_merge<KNN_U8>, dim3(ns), dim3(MT), 0, st, slots, X, B, G);
    else
      hipLaunchKernelGGL(k_cand_merge<KNN_F32>, dim3(ns), dim3(MT), 0, st, slots, X, B, G);
    prof_end(tok, st, 0.0);
  }
  tok = prof_begin(PROF_SELECT, st);
  hipLaunchKernelGGL(k_select_partial, dim3((unsigned)((G.n + SEL_CH - 1) / SEL_CH), ns), dim3(NT), 0, st, slots,
                     B, G);
  hipLaunchKernelGGL(k_select_merge, dim3(ns), dim3(MT), 0, st, slots, B, G, 0);
  prof_end(tok, st, 0.0);
  tok = prof_begin(PROF_DECIDE, st);
  hipLaunchKernelGGL(k_decide, dim3((unsigned)((G.n + DEC_CH - 1) / DEC_CH), ns), dim3(NT), 0, st, slots,
                     B, G);
  prof_end(tok, st, 0.0);
  tok = prof_begin(PROF_FINISH, st);
  if (G.dtype == KNN_U8)
    hipLaunchKernelGGL(k_finish<KNN_U8>, dim3(ns), dim3(MT), 0, st, slots, qd, sched, ctl, X, B, G, 0);
  else
    hipLaunchKernelGGL(k_finish<KNN_F32>, dim3(ns), dim3(MT), 0, st, slots, qd, sched, ctl, X, B, G, 0);
  if (G.packed_admit)
    hipLaunchKernelGGL(k_admit_packed, dim3(1), dim3(MT), 0, st, slots, qd, sched, ctl, G.n, G.m, G.nslots_all);
  prof_end(tok, st, 0.0);
}

void launch_admit(Slot *slots, const QDesc *qd, const Sched *sched, Ctl *ctl, const uint8_t *X, const Bufs &B,
                  const Geometry &G, hipStream_t st, bool direct) {
  const unsigned ns = (unsigned)G.nslots;
  const int mode = direct ? 2 : 1;
  if (G.dtype == KNN_U8)
    hipLaunchKernelGGL(k_finish<KNN_U8>, dim3(ns), dim3(MT), 0, st, slots, qd, sched, ctl, X, B, G, mode);
  else
    hipLaunchKernelGGL(k_finish<KNN_F32>, dim3(ns), dim3(MT), 0, st, slots, qd, sched, ctl, X, B, G, mode);
}

int64_t part_words(int64_t n, int32_t kmax, int32_t cmax) {
  int64_t nsel = (n + SEL_CH - 1) / SEL_CH;
  if (kmax + 1 <= kPmMaxK1) nsel = std::max<int64_t>(nsel, (n + FS_PT - 1) / FS_PT);  // point-major selection
  const int64_t ncand = (n + CAND_CH - 1) / CAND_CH;
  int64_t a = nsel * (2 * (int64_t)kmax + 1);
  a = std::max<int64_t>(a, (3 * ((n + DQ_PT - 1) / DQ_PT) + 1) / 2);  // k_decide_pm's count records (u32 triples)
  const int64_t c = cmax > 0 ? ncand * (int64_t)min(cmax, CAND_CH) * 2 : 0;  // keys + packed ids
  return (a > c ? a : c) + fs_mixed_words(n) + 8;  // the mixed-tile list of k_select_pm at the end
}

}  // namespace knn
