// k_naive_f32.hip -- the naive scan of Section 3 for float data on the
// matrix cores, returning exactly the set (and distances) of an FP64 scan.
//
// 1. Split BF16: every value v is stored as hi = bf16(v), lo = bf16(v - hi),
//    so |v - hi - lo| <= 2^-16 |v|.  The dot product q.x is taken as
//    hi.hi + hi.lo + lo.hi with v_mfma_f32_16x16x32_bf16 (three MFMAs per
//    k-step, fp32 accumulation), and the distance as |q|^2 + |x|^2 - 2 q.x.
// 2. Error bound per pair: |d~ - d| <= E = c1 |q| |x| + c2 (|q|^2 + |x|^2),
//    c1 covering the split (3.01 2^-16 per product) and fp32 accumulation of
//    3m terms (3m 2^-24), doubled for safety; c2 the fp32 epilogue roundings.
// 3. A probe over the first tiles of every point range keeps, per query and
//    range, the k smallest upper bounds u = d~ + E of the points it sees
//    (in a wave register, lane j the j-th smallest, fed through a small LDS
//    buffer).  tau0, the k-th smallest u over the union of those lists, is
//    the upper bound of k real points, so tau0 >= d_(k); every true k-NN
//    point has l = d~ - E <= d <= d_(k) <= tau0.
// 4. The full scan screens each pair in the MFMA fragment layout and
//    appends the pairs with l <= tau0 to the (query, range) candidate list;
//    over a probe of s of the n points about k n / s points lie below tau0.
//    A list that overflows its capacity sends its query to an exact rescan.
// 5. The candidates are rescored in FP64, summing (x_j - q_j)^2 in
//    coordinate order like the CPU reference, and the k smallest by
//    (distance, index) are returned.
// The l1 distance has no product form: its tile sums |x_j - q_j| in fp32 on
// the vector ALUs from zero-padded rows (each lane adds its pairs' terms in
// coordinate order), with the relative bound |d~ - d| <= c1 d~ (m terms,
// each rounded twice: c1 = 2 (m + 2) 2^-24, doubled for safety), and the same
// candidate lists, completeness check and FP64 rescoring (sum of |x_j - q_j|).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "block_select.h"
#include "knn_host.h"
#include "knn_prof.h"

namespace knn {

typedef int v4i_f __attribute__((ext_vector_type(4)));
typedef float v4f_f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf_f __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t bf16_rne(float v) {
  const uint32_t b = __float_as_uint(v);
  return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// order-preserving 32-bit key of a float
__device__ __forceinline__ uint32_t fkey(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float fkey_inv(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Rows of a float matrix -> split BF16 (hi, lo) padded to mp, |row|^2 (fp64
// sum rounded to fp32) and |row|.
__global__ __launch_bounds__(256) void k_split_rows(const float *__restrict__ A, int64_t rows, int64_t m,
                                                    int64_t mp, uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                                                    float *__restrict__ nrm, float *__restrict__ rn) {
  const int64_t r = blockIdx.x;
  if (r >= rows) return;
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < mp; j += 256) {
    const float v = j < m ? A[r * m + j] : 0.0f;
    const uint16_t h = bf16_rne(v);
    const uint16_t l = bf16_rne(v - bf16_to_f(h));
    hi[r * mp + j] = h;
    lo[r * mp + j] = l;
    acc += (double)v * (double)v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = red[0] + red[1] + red[2] + red[3];
    nrm[r] = (float)t;
    rn[r] = (float)sqrt(t);
  }
}

constexpr int FBQ = 64, FBP = 128, FROWB = 80, FDSTR = FBP + 4;
constexpr int KCU = 64;   // upper-bound list capacity (k <= 64): one wave register per query
constexpr int FCB = 16;   // buffered upper-bound candidates per query before a merge
constexpr int FCL = 384;  // candidate list capacity per (query, range)

constexpr int64_t FPROBE = 1;         // at least this many tiles of every range in the probe pass
constexpr int64_t FPROBE_PTS = 32768;  // and at least this many points in all

// Per query: the k-th smallest of the ranges' upper-bound lists (a key of
// a real point's upper bound, so >= d_(k)) lowers the shared bound.
__global__ __launch_bounds__(256) void k_naive_f32_tau0(const uint64_t *__restrict__ part, int64_t nranges, int k,
                                                        uint32_t *__restrict__ gtau) {
  const int64_t q = blockIdx.x;
  const uint64_t *pq = part + q * nranges * k;
  __shared__ SelScratch ss;
  int less;
  const uint64_t v = block_kth_gen<256>(nranges * k, [&](int64_t t) { return pq[t]; }, k, ss, &less);
  if (threadIdx.x == 0 && v != ~0ull) atomicMin(&gtau[q], (uint32_t)(v >> 32));
}

__global__ void k_fill_u32(uint32_t *__restrict__ a, int64_t len, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// SCREEN = false: the probe (the k smallest upper bounds per query over
// the first max_tiles tiles of each range, kept in a wave register per
// query); true: the screen pass, with every query's bound fixed
// beforehand in gtau -- the candidates are the pairs whose lower bound is
// at or below it, and nothing else is kept.
template <int MET, bool SCREEN>
__global__ __launch_bounds__(256) void k_naive_f32(const uint16_t *__restrict__ Qh, const uint16_t *__restrict__ Ql,
                                                   const float *__restrict__ qn, const float *__restrict__ qr,
                                                   const uint16_t *__restrict__ Xh, const uint16_t *__restrict__ Xl,
                                                   const float *__restrict__ xn, const float *__restrict__ xr,
                                                   int64_t nq, int64_t n, int64_t mp, int k, int64_t prange,
                                                   float c1, float c2, uint64_t *__restrict__ part,
                                                   uint64_t *__restrict__ cand, int32_t *__restrict__ ncand,
                                                   int64_t nranges, uint32_t *__restrict__ gtau, int64_t max_tiles) {
  constexpr uint64_t PAD = ~0ull;
  constexpr int QPW = FBQ / 4;  // queries owned by one wave in the epilogue
  __shared__ __align__(16) uint8_t tiles[FBQ * FDSTR * 4];
  static_assert(2 * (FBQ + FBP) * FROWB <= FBQ * FDSTR * 4, "tile union too small");
  uint8_t *Ah = tiles, *Al = tiles + FBQ * FROWB;
  uint8_t *Bh = tiles + 2 * FBQ * FROWB, *Bl = Bh + FBP * FROWB;
  float *Ds = reinterpret_cast<float *>(tiles);
  __shared__ uint64_t Cb[SCREEN ? 1 : FBQ][FCB];  // (the screen pass keeps no lists)
  // per query of the block: its sorted upper-bound list (entry j the j-th
  // smallest, PAD while fewer than k), the count of its LDS buffer and of
  // its candidate list in this range, and its norms
  __shared__ uint64_t Lq[SCREEN ? 1 : FBQ][kWave];
  __shared__ uint64_t tauq[FBQ];  // entry k - 1 of the query's list
  __shared__ __align__(16) float tauf[FBQ];  // the same as a float (+inf while the list holds fewer than k)
  __shared__ int cbq[FBQ], ncq[FBQ];
  __shared__ __align__(16) float qnq[FBQ], qrq[FBQ];
  __shared__ uint8_t qflag[FBQ];       // the query has a pair in this tile that passes the screen
  __shared__ __align__(16) float gtf[FBQ];  // the screen pass's fixed bound per query
  __shared__ float txn[FBP], txr[FBP];  // the tile's point norms
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int64_t q0 = (int64_t)blockIdx.y * FBQ;
  const int64_t pr0 = (int64_t)blockIdx.x * prange;
  const int64_t pr1 = std::min(std::min(n, pr0 + prange), pr0 + max_tiles * FBP);  // (a probe pass: its first tiles)
  const int wq = wave >> 1, wp = wave & 1;
  if (!SCREEN)
    for (int j = tid; j < FBQ * kWave; j += 256) Lq[j / kWave][j % kWave] = PAD;
  if (tid < FBQ) {
    const int64_t q = q0 + tid;
    tauq[tid] = PAD;
    tauf[tid] = INFINITY;
    gtf[tid] = INFINITY;
    qflag[tid] = 0;
    cbq[tid] = 0;
    ncq[tid] = 0;
    qnq[tid] = (MET == KNN_METRIC_L1 || q >= nq) ? 0.0f : qn[q];
    qrq[tid] = (MET == KNN_METRIC_L1 || q >= nq) ? 0.0f : qr[q];
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  // the fragment layout's queries of this lane: 32 wq + 16 a + 4 (lane >> 4) + v
  float qnf[2][4], cqr[2][4];  // |q|^2 and c1 |q| (squared l2)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ql = 32 * wq + 16 * a + 4 * (lane >> 4) + v;
      qnf[a][v] = qnq[ql];
      cqr[a][v] = c1 * qrq[ql];
    }
  // squared l2: the next 64-byte K slice of the tile's query and point rows
  // (hi and lo), loaded into registers one slice ahead
  v4i_f pah = v4i_f{0, 0, 0, 0}, pal = v4i_f{0, 0, 0, 0}, pbh[2], pbl[2];
  auto fetch = [&](int64_t pt, int64_t k0) {
    {
      const int r = tid >> 2, c = (tid & 3) * 16;
      pah = v4i_f{0, 0, 0, 0};
      pal = v4i_f{0, 0, 0, 0};
      if (q0 + r < nq) {
        pah = *reinterpret_cast<const v4i_f *>(reinterpret_cast<const uint8_t *>(Qh + (q0 + r) * mp + k0) + c);
        pal = *reinterpret_cast<const v4i_f *>(reinterpret_cast<const uint8_t *>(Ql + (q0 + r) * mp + k0) + c);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = (tid >> 2) + 64 * h, c = (tid & 3) * 16;
      pbh[h] = v4i_f{0, 0, 0, 0};
      pbl[h] = v4i_f{0, 0, 0, 0};
      if (pt + r < pr1) {
        pbh[h] = *reinterpret_cast<const v4i_f *>(reinterpret_cast<const uint8_t *>(Xh + (pt + r) * mp + k0) + c);
        pbl[h] = *reinterpret_cast<const v4i_f *>(reinterpret_cast<const uint8_t *>(Xl + (pt + r) * mp + k0) + c);
      }
    }
  };
  if constexpr (MET != KNN_METRIC_L1) {
    if (pr0 < pr1) fetch(pr0, 0);
  }
  if (SCREEN && tid < FBQ && q0 + tid < nq) {  // (fixed for the whole pass)
    const uint32_t g = gtau[q0 + tid];
    gtf[tid] = g == ~0u ? INFINITY : fkey_inv(g);
  }
  for (int64_t p0 = pr0; p0 < pr1; p0 += FBP) {
    if (!SCREEN && tid < FBQ && q0 + tid < nq) {
      // probe: the smallest running bound any range of the query has
      // published; the union's k-th smallest upper bound lies at or below
      // it, so a pair whose upper bound exceeds it cannot change the result
      // (read by this tile's screen, after the K loop's barriers)
      const uint32_t g = __hip_atomic_load(&gtau[q0 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      gtf[tid] = g == ~0u ? INFINITY : fkey_inv(g);
    }
    // this lane's four points of the fragment layout (64 wp + 16 b + (lane &
    // 15)): norms loaded before the K loop so that their latency is hidden
    float xnf[4] = {0.0f, 0.0f, 0.0f, 0.0f}, xrf[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (MET != KNN_METRIC_L1) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t p = p0 + 64 * wp + 16 * b + (lane & 15);
        if (p < pr1) {
          xnf[b] = xn[p];
          xrf[b] = xr[p];
        }
      }
    }
    v4f_f acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = v4f_f{0.f, 0.f, 0.f, 0.f};
    if constexpr (MET == KNN_METRIC_L1) {
      // Qh / Xh hold zero-padded f32 rows here; 16 floats = 64 bytes per row per step
      const float *Qf = reinterpret_cast<const float *>(Qh), *Xf = reinterpret_cast<const float *>(Xh);
      for (int64_t k0 = 0; k0 < mp; k0 += 16) {
        {
          const int r = tid >> 2, c = (tid & 3) * 4;
          v4f_f v = v4f_f{0.f, 0.f, 0.f, 0.f};
          if (q0 + r < nq) v = *reinterpret_cast<const v4f_f *>(Qf + (q0 + r) * mp + k0 + c);
          *reinterpret_cast<v4f_f *>(Ah + r * FROWB + 4 * c) = v;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int r = (tid >> 2) + 64 * h, c = (tid & 3) * 4;
          v4f_f v = v4f_f{0.f, 0.f, 0.f, 0.f};
          if (p0 + r < pr1) v = *reinterpret_cast<const v4f_f *>(Xf + (p0 + r) * mp + k0 + c);
          *reinterpret_cast<v4f_f *>(Bh + r * FROWB + 4 * c) = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
          v4f_f qv[2][4], pv[4];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              qv[a][v] = *reinterpret_cast<const v4f_f *>(Ah + (32 * wq + 16 * a + 4 * (lane >> 4) + v) * FROWB + 4 * kk);
#pragma unroll
          for (int b = 0; b < 4; ++b)
            pv[b] = *reinterpret_cast<const v4f_f *>(Bh + (64 * wp + 16 * b + (lane & 15)) * FROWB + 4 * kk);
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                float t = acc[a][b][v];
#pragma unroll
                for (int e = 0; e < 4; ++e) t += fabsf(qv[a][v][e] - pv[b][e]);
                acc[a][b][v] = t;
              }
        }
        __syncthreads();
      }
    } else
    for (int64_t k0 = 0; k0 < mp; k0 += 32) {  // 32 bf16 = 64 bytes per row per step
      // the prefetched slice into LDS, then the next one's loads (this
      // tile's next slice, or the next tile's first) in flight while this
      // one is consumed -- and, for a tile's last slice, during the epilogue
      {
        const int r = tid >> 2, c = (tid & 3) * 16;
        *reinterpret_cast<v4i_f *>(Ah + r * FROWB + c) = pah;
        *reinterpret_cast<v4i_f *>(Al + r * FROWB + c) = pal;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = (tid >> 2) + 64 * h, c = (tid & 3) * 16;
        *reinterpret_cast<v4i_f *>(Bh + r * FROWB + c) = pbh[h];
        *reinterpret_cast<v4i_f *>(Bl + r * FROWB + c) = pbl[h];
      }
      __syncthreads();
      if (k0 + 32 < mp)
        fetch(p0, k0 + 32);
      else if (p0 + FBP < pr1)
        fetch(p0 + FBP, 0);
      v8bf_f ah[2], al[2], bh[4], bl[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int off = (32 * wq + 16 * a + (lane & 15)) * FROWB + 16 * (lane >> 4);
        ah[a] = *reinterpret_cast<const v8bf_f *>(Ah + off);
        al[a] = *reinterpret_cast<const v8bf_f *>(Al + off);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int off = (64 * wp + 16 * b + (lane & 15)) * FROWB + 16 * (lane >> 4);
        bh[b] = *reinterpret_cast<const v8bf_f *>(Bh + off);
        bl[b] = *reinterpret_cast<const v8bf_f *>(Bl + off);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        }
      __syncthreads();
    }
    // Screen in the fragment layout.  Screen pass: a pair is a candidate
    // when its lower bound l = d~ - E is at or below the query's fixed
    // bound, and is appended at once.  Probe: a pair can enter the query's
    // list only when its upper bound d~ + E is at or below the running one;
    // the expressions are the per-query pass's own, so the flag is a
    // superset of its condition, and queries with no such pair in the tile
    // are skipped there (they would change nothing).
    bool anyq = false;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int ql0 = 32 * wq + 16 * a + 4 * (lane >> 4);
      // (screen pass: the fixed bound; probe: the smaller of the query's
      // running bound here and the smallest any range has published)
      const v4f_f tg = *reinterpret_cast<const v4f_f *>(&gtf[ql0]);
      v4f_f tq = tg;
      if constexpr (!SCREEN) {
        const v4f_f tl = *reinterpret_cast<const v4f_f *>(&tauf[ql0]);
        tq = v4f_f{fminf(tl[0], tg[0]), fminf(tl[1], tg[1]), fminf(tl[2], tg[2]), fminf(tl[3], tg[3])};
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        bool f = false;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int64_t p = p0 + 64 * wp + 16 * b + (lane & 15);
          const float dot = acc[a][b][v];
          // the screen pass tests the lower bound (a candidate), the probe
          // the upper bound (an insertion into the running list)
          float bnd;
          if constexpr (MET == KNN_METRIC_L1) {
            bnd = SCREEN ? dot - c1 * dot : dot + c1 * dot;
          } else {
            const float sn = qnf[a][v] + xnf[b];
            const float d = sn - 2.0f * dot;
            const float E = cqr[a][v] * xrf[b] + c2 * sn;
            bnd = SCREEN ? d - E : d + E;
          }
          const float lo = bnd;
          const bool pass = p < pr1 && q0 + ql0 + v < nq && bnd <= tq[v];  // (padding queries of the last tile: none)
          if constexpr (SCREEN) {
            if (pass) {  // a candidate: appended to the query's list of this range
              const int ql = ql0 + v;
              const int pos = atomicAdd(&ncq[ql], 1);
              if (pos < FCL) cand[((q0 + ql) * nranges + blockIdx.x) * (int64_t)FCL + pos] =
                  ((uint64_t)fkey(lo) << 32) | (uint64_t)p;
            }
          }
          f |= pass;
        }
        if constexpr (!SCREEN) {
          const uint64_t mk = __ballot(f);
          if ((lane & 15) == 0 && ((mk >> (lane & 48)) & 0xFFFFull) != 0) qflag[ql0 + v] = 1;
          anyq |= mk != 0;
        }
      }
    }
    if constexpr (SCREEN) continue;  // (the next tile's first LDS writes follow the K loop's last barrier)
    if ((lane >> 4) == 0) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int pl = 64 * wp + 16 * b + lane;
        txn[pl] = xnf[b];
        txr[pl] = xrf[b];
      }
    }
    if (__syncthreads_or(anyq ? 1 : 0) == 0) continue;  // (block-uniform) nothing in this tile for any query
    // the tile's sums (dot products, or l1 sums) as [query][point] rows
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ql = 32 * wq + 16 * a + 4 * (lane >> 4) + v;
          const int pl = 64 * wp + 16 * b + (lane & 15);
          Ds[ql * FDSTR + pl] = acc[a][b][v];
        }
    __syncthreads();
    // per flagged query of this wave: upper bounds below the running k-th
    // one go to the LDS buffer (merged into the list when it would
    // overflow)
#pragma unroll 1
    for (int t = 0; t < QPW; ++t) {
      const int ql = wave * QPW + t;
      const int64_t q = q0 + ql;
      if (q >= nq) break;  // (wave-uniform)
      if (!qflag[ql]) continue;
      const float qnv = qnq[ql], qrv = qrq[ql];
      uint64_t cu[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int pl = lane + 64 * h;
        const int64_t p = p0 + pl;
        cu[h] = PAD;
        if (p < pr1) {
          const float dot = Ds[ql * FDSTR + pl];
          const float xnv = txn[pl], xrv = txr[pl];
          const float d = MET == KNN_METRIC_L1 ? dot : (qnv + xnv) - 2.0f * dot;
          const float E = MET == KNN_METRIC_L1 ? c1 * d : c1 * qrv * xrv + c2 * (qnv + xnv);
          cu[h] = ((uint64_t)fkey(d + E) << 32) | (uint64_t)p;
        }
      }
      uint64_t tau = tauq[ql];
      if (tau == PAD) {
        // until the list holds k upper bounds, this tile's go straight into
        // it, so that the bound below is finite from the first tile on
        const int cb = cbq[ql];
        uint64_t L = Lq[ql][lane];
        if (cb > 0) L = merge_sorted64(L, lane < cb ? Cb[ql][lane] : PAD);
        L = merge_sorted64(L, cu[0]);
        L = merge_sorted64(L, cu[1]);
        cu[0] = PAD;
        cu[1] = PAD;
        Lq[ql][lane] = L;
        tau = wave_bcast_u64(L, k - 1);
        if (lane == 0) {
          cbq[ql] = 0;
          tauq[ql] = tau;
          tauf[ql] = tau == PAD ? INFINITY : fkey_inv((uint32_t)(tau >> 32));
          if (tau != PAD) atomicMin(&gtau[q], (uint32_t)(tau >> 32));
        }
      }
      // tau: the k-th smallest upper bound of the points seen so far (the
      // buffered ones left out)
      const bool a0 = cu[0] < tau, a1 = cu[1] < tau;
      const uint64_t u0 = __ballot(a0), u1 = __ballot(a1);
      if (u0 | u1) {  // (wave-uniform) upper bounds below tau
        const int n0 = __popcll(u0), n1 = __popcll(u1);
        const int cb = cbq[ql];
        if (cb + n0 + n1 > FCB) {
          // does not fit: the buffer (written in earlier tiles, before the
          // last barrier) and this tile's candidates merge into the list
          uint64_t L = Lq[ql][lane];
          if (cb > 0) L = merge_sorted64(L, lane < cb ? Cb[ql][lane] : PAD);
          L = merge_sorted64(L, a0 ? cu[0] : PAD);
          L = merge_sorted64(L, a1 ? cu[1] : PAD);
          Lq[ql][lane] = L;
          const uint64_t nt = wave_bcast_u64(L, k - 1);
          if (lane == 0) {
            cbq[ql] = 0;
            tauq[ql] = nt;
            tauf[ql] = nt == PAD ? INFINITY : fkey_inv((uint32_t)(nt >> 32));
            if (nt != PAD) atomicMin(&gtau[q], (uint32_t)(nt >> 32));
          }
        } else {
          if (a0) Cb[ql][cb + __popcll(u0 & lt)] = cu[0];
          if (a1) Cb[ql][cb + n0 + __popcll(u1 & lt)] = cu[1];
          if (lane == 0) cbq[ql] = cb + n0 + n1;
        }
      }
      if (lane == 0) qflag[ql] = 0;
    }
    __syncthreads();
  }
  __syncthreads();  // (the screen pass's appends counted)
  // final merge; per query the range's k smallest upper bounds and the
  // length of its candidate list
#pragma unroll 1
  for (int t = 0; t < QPW; ++t) {
    const int ql = wave * QPW + t;
    const int64_t q = q0 + ql;
    if (q >= nq) break;
    if (SCREEN) {
      if (lane == 0) ncand[q * nranges + blockIdx.x] = ncq[ql];
      continue;
    }
    uint64_t L = Lq[ql][lane];
    const int cb = cbq[ql];
    if (cb > 0) L = merge_sorted64(L, lane < cb ? Cb[ql][lane] : PAD);
    if (lane < k) part[(q * nranges + blockIdx.x) * (int64_t)k + lane] = L;
    if (lane == 0) ncand[q * nranges + blockIdx.x] = ncq[ql];
  }
}

// Exact FP64 distance of point i (squared l2 or l1), coordinates in order
// (no FMA contraction).
__device__ __forceinline__ double exact_f64(const float *__restrict__ X, const float *__restrict__ q, int64_t m,
                                            int64_t i, int met) {
  const float *row = X + i * m;
  double s = 0.0;
  if (met == KNN_METRIC_L1) {
    for (int64_t j = 0; j < m; ++j) s += fabs((double)row[j] - (double)q[j]);
    return s;
  }
  for (int64_t j = 0; j < m; ++j) {
    const double d = (double)row[j] - (double)q[j];
    s += d * d;
  }
  return s;
}

constexpr int FCAP = 2048;  // candidate capacity per query in the merge
constexpr int FMT = 1024;   // threads of a merge block (one candidate each while rescoring)
constexpr int FROWS = 12288;  // floats of LDS for candidate rows staged by the merge (48 KB)
constexpr int FRANGES = 1024;  // point ranges whose lists the merge enumerates by prefix sums

// The same sum over a row staged in LDS (stride >= m) and the query in LDS.
__device__ __forceinline__ double exact_f64_lds(const float *row, const float *q, int64_t m, int met) {
  double s = 0.0;
  if (met == KNN_METRIC_L1) {
    for (int64_t j = 0; j < m; ++j) s += fabs((double)row[j] - (double)q[j]);
    return s;
  }
  for (int64_t j = 0; j < m; ++j) {
    const double d = (double)row[j] - (double)q[j];
    s += d * d;
  }
  return s;
}

__global__ __launch_bounds__(FMT) void k_naive_f32_merge(const uint64_t *__restrict__ candl,
                                                          const int32_t *__restrict__ ncand, int64_t nranges, int k,
                                                          const float *__restrict__ X, const float *__restrict__ Q,
                                                          int64_t m, int met, int64_t *__restrict__ out_idx,
                                                          double *__restrict__ out_dist, int32_t *__restrict__ flag,
                                                          const uint32_t *__restrict__ gtau) {
  const int64_t q = blockIdx.x;
  __shared__ uint64_t key[FCAP];
  __shared__ int32_t id[FCAP];
  __shared__ int cnt, bad;
  // the screen pass's bound (>= d_(k)); every candidate lies at or below it
  const float tau = gtau[q] == ~0u ? INFINITY : fkey_inv(gtau[q]);
  const uint32_t tau_key = fkey(tau + fabsf(tau) * 1e-6f + 1e-30f);  // tiny margin over fp32 rounding
  if (threadIdx.x == 0) {
    cnt = 0;
    bad = 0;
  }
  __syncthreads();
  // a range whose candidate list overflowed may have dropped a candidate;
  // the lists' lengths, then their entries enumerated through the prefix
  // sums of the lengths (ranges at most FRANGES here, else range by range)
  __shared__ int32_t pre[FRANGES + 1];
  for (int64_t r = threadIdx.x; r < nranges; r += FMT)
    if (ncand[q * nranges + r] > FCL) atomicOr(&bad, 1);
  const bool small = nranges <= FRANGES;
  if (small && threadIdx.x == 0) {
    int acc = 0;
    for (int64_t r = 0; r < nranges; ++r) {
      pre[r] = acc;
      acc += min(ncand[q * nranges + r], FCL);
    }
    pre[nranges] = acc;
  }
  __syncthreads();
  auto take = [&](uint64_t e) {
    if ((uint32_t)(e >> 32) <= tau_key) {
      const int pos = atomicAdd(&cnt, 1);
      if (pos < FCAP) id[pos] = (int32_t)(e & 0xFFFFFFFFu);
      else atomicOr(&bad, 1);
    }
  };
  if (!bad && small) {
    for (int t = threadIdx.x; t < pre[nranges]; t += FMT) {
      int lo = 0, hi = (int)nranges;  // the range r with pre[r] <= t < pre[r + 1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (pre[mid] <= t) lo = mid;
        else hi = mid;
      }
      take(candl[(q * nranges + lo) * FCL + (t - pre[lo])]);
    }
  } else if (!bad) {
    for (int64_t t = threadIdx.x; t < nranges * FCL; t += FMT) {
      const int64_t r = t / FCL, j = t % FCL;
      if (j >= ncand[q * nranges + r]) continue;
      take(candl[(q * nranges + r) * FCL + j]);
    }
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) flag[q] = 1;
    return;
  }
  const int c = cnt;
  const float *qv = Q + q * m;
  // Rescoring, each candidate's sum in coordinate order by one thread.  For
  // short rows the candidates' rows are staged in LDS a batch at a time by
  // coalesced loads (rows padded to an odd stride: one bank per thread),
  // the query too; long rows are read from global memory directly.
  __shared__ float rows[FROWS];
  const int64_t stride = m | 1;
  const int nb = (int)std::min<int64_t>(FMT, (FROWS - stride) / stride);  // (one stride for the query)
  if (nb >= 32) {
    float *qs = rows + (int64_t)nb * stride;
    for (int64_t j = threadIdx.x; j < m; j += FMT) qs[j] = qv[j];
    for (int c0 = 0; c0 < c; c0 += nb) {
      const int cb = std::min(nb, c - c0);
      __syncthreads();  // (the previous batch's rows are consumed)
      for (int64_t e = threadIdx.x; e < (int64_t)cb * m; e += FMT) {
        const int64_t r = e / m, j = e - r * m;
        rows[r * stride + j] = X[(int64_t)id[c0 + r] * m + j];
      }
      __syncthreads();
      if (threadIdx.x < cb) key[c0 + threadIdx.x] = dkey(exact_f64_lds(rows + threadIdx.x * stride, qs, m, met));
    }
  } else {
    for (int t = threadIdx.x; t < c; t += FMT) key[t] = dkey(exact_f64(X, qv, m, id[t], met));
  }
  __syncthreads();
  int len = 1;
  while (len < c) len <<= 1;
  for (int t = c + (int)threadIdx.x; t < len; t += FMT) {
    key[t] = ~0ull;
    id[t] = 0x7FFFFFFF;
  }
  block_bitonic_sort<FMT>(key, id, len);
  for (int t = threadIdx.x; t < k; t += FMT) {
    out_idx[q * k + t] = t < c ? (int64_t)id[t] : -1;
    if (out_dist) out_dist[q * k + t] = t < c ? dkey_inv(key[t]) : INFINITY;
  }
  if (threadIdx.x == 0) flag[q] = 0;
}

// Exact FP64 scan of one query (used when a candidate list may be incomplete).
__global__ __launch_bounds__(1024) void k_naive_f32_full(const float *__restrict__ X, const float *__restrict__ Q,
                                                         int64_t n, int64_t m, int met, int k,
                                                         const int32_t *__restrict__ qids,
                                                         double *__restrict__ scratch, int64_t *__restrict__ out_idx,
                                                         double *__restrict__ out_dist) {
  const int64_t q = qids[blockIdx.x];
  double *dd = scratch + (int64_t)blockIdx.x * n;
  const float *qv = Q + q * m;
  for (int64_t i = threadIdx.x; i < n; i += 1024) dd[i] = exact_f64(X, qv, m, i, met);
  __syncthreads();
  __shared__ SelScratch ss;
  __shared__ uint64_t key[kMaxKH];
  __shared__ int32_t id[kMaxKH];
  __shared__ int cnt;
  int less;
  const uint64_t v = block_kth_gen<1024>(n, [&](int64_t i) { return dkey(dd[i]); }, k, ss, &less);
  const uint32_t thr = block_kth_u32_gen<1024>(
      n, [&](int64_t i) { return (uint32_t)i; }, [&](int64_t i) { return dkey(dd[i]) == v; }, k - less, ss);
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const uint64_t kk = dkey(dd[i]);
    if (kk < v || (kk == v && (uint32_t)i <= thr)) {
      const int pos = atomicAdd(&cnt, 1);
      if (pos < kMaxKH) {
        key[pos] = kk;
        id[pos] = (int32_t)i;
      }
    }
  }
  __syncthreads();
  int len = 1;
  while (len < k) len <<= 1;
  for (int t = k + (int)threadIdx.x; t < len; t += 1024) {
    key[t] = ~0ull;
    id[t] = 0x7FFFFFFF;
  }
  block_bitonic_sort<1024>(key, id, len);
  for (int t = threadIdx.x; t < k; t += 1024) {
    out_idx[q * k + t] = (int64_t)id[t];
    if (out_dist) out_dist[q * k + t] = dkey_inv(key[t]);
  }
}

int naive_prepare_db_f32(knn_db_s *db, hipStream_t st) {
  const size_t cells = (size_t)db->n * db->mp;
  HIP_TRY(hipMalloc(&db->xbf, cells * 2 * sizeof(uint16_t)));  // hi, then lo
  HIP_TRY(hipMalloc(&db->norm_f, sizeof(float) * db->n));
  HIP_TRY(hipMalloc(&db->rownorm, sizeof(float) * db->n));
  hipLaunchKernelGGL(k_split_rows, dim3((unsigned)db->n), dim3(256), 0, st, (const float *)db->X, db->n, db->m,
                     db->mp, db->xbf, db->xbf + cells, db->norm_f, db->rownorm);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return KNN_OK;
}

// Exact FP64 scans of the listed queries (k_naive_f32_full), as many per
// launch as 1 GiB of distance scratch holds.
static int exact_f32_queries(knn_db_s *db, const float *dq, const std::vector<int32_t> &ids, int32_t k,
                             int64_t *out_idx, double *out_dist, hipStream_t st) {
  if (ids.empty()) return KNN_OK;
  const int64_t n = db->n, m = db->m;
  const int64_t batch = std::max<int64_t>(1, std::min<int64_t>((int64_t)ids.size(), (1ll << 30) / (n * 8)));
  int32_t *dq_ids = nullptr;
  double *scratch = nullptr;
  HIP_TRY(hipMallocAsync(&dq_ids, sizeof(int32_t) * ids.size(), st));
  HIP_TRY(hipMallocAsync(&scratch, sizeof(double) * n * batch, st));
  HIP_TRY(hipMemcpyAsync(dq_ids, ids.data(), sizeof(int32_t) * ids.size(), hipMemcpyHostToDevice, st));
  for (int64_t b0 = 0; b0 < (int64_t)ids.size(); b0 += batch) {
    const int64_t cnt = std::min<int64_t>(batch, (int64_t)ids.size() - b0);
    hipLaunchKernelGGL(k_naive_f32_full, dim3((unsigned)cnt), dim3(1024), 0, st, (const float *)db->X, dq, n, m,
                       db->metric, k, dq_ids + b0, scratch, out_idx, out_dist);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipFreeAsync(scratch, st));
  HIP_TRY(hipFreeAsync(dq_ids, st));
  HIP_TRY(hipStreamSynchronize(st));  // (the host list is freed on return)
  return KNN_OK;
}

int naive_f32(knn_db_s *db, const float *dq, int64_t nq, int32_t k, int64_t *out_idx, double *out_dist,
              hipStream_t st) {
  if (k > KCU) {  // above the upper-bound lists' capacity: every query scanned exactly in FP64
    std::vector<int32_t> all((size_t)nq);
    for (int64_t q = 0; q < nq; ++q) all[(size_t)q] = (int32_t)q;
    return exact_f32_queries(db, dq, all, k, out_idx, out_dist, st);
  }
  const bool l1 = db->metric == KNN_METRIC_L1;
  const int64_t n = db->n, m = db->m, mp = db->mp;
  const size_t cells = (size_t)n * mp;
  const int64_t qt = (nq + FBQ - 1) / FBQ;
  int64_t prange = (n * qt + 1023) / 1024;
  prange = std::max<int64_t>(FBP, (prange + FBP - 1) / FBP * FBP);
  const int64_t nranges = (n + prange - 1) / prange;
  // error-bound constants (doubled for safety, see the file header)
  const double u16 = 1.0 / 65536.0, u24 = 1.0 / 16777216.0;
  const float c1 = l1 ? (float)(2.0 * ((double)m + 2.0) * u24) : (float)(2.0 * 2.0 * (3.01 * u16 + 3.1 * (double)m * u24));
  const float c2 = (float)(8.0 * u24);
  const size_t b_qs = (size_t)nq * mp * 2 * 2, b_qn = sizeof(float) * nq * 2 + 512,
               b_part = sizeof(uint64_t) * nq * nranges * k + 256,
               b_cand = sizeof(uint64_t) * nq * nranges * FCL, b_nc = sizeof(int32_t) * nq * nranges + 256,
               b_flag = sizeof(int32_t) * nq + 256, b_gtau = sizeof(uint32_t) * nq + 256;
  void *ws = nullptr;
  HIP_TRY(hipMallocAsync(&ws, b_qs + b_qn + b_part + b_cand + b_nc + b_flag + b_gtau, st));
  uint16_t *Qh = (uint16_t *)ws, *Ql = Qh + (size_t)nq * mp;
  float *qn = (float *)((uint8_t *)ws + b_qs), *qr = qn + nq;
  uint64_t *part = (uint64_t *)((uint8_t *)ws + b_qs + b_qn);
  uint64_t *candl = (uint64_t *)((uint8_t *)ws + b_qs + b_qn + b_part);
  int32_t *ncand = (int32_t *)((uint8_t *)ws + b_qs + b_qn + b_part + b_cand);
  int32_t *flag = (int32_t *)((uint8_t *)ws + b_qs + b_qn + b_part + b_cand + b_nc);
  uint32_t *gtau = (uint32_t *)((uint8_t *)ws + b_qs + b_qn + b_part + b_cand + b_nc + b_flag);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((nq + 255) / 256, 1024)), dim3(256), 0, st, gtau, nq,
                     ~0u);
  int tok = prof_begin(PROF_NAIVE_REST, st);
  if (l1)  // zero-padded f32 query rows (nq x mp x 4 bytes, the size of the split pair)
    launch_pad_rows(reinterpret_cast<const uint8_t *>(dq), nq, m, mp, 4, reinterpret_cast<uint8_t *>(Qh), st);
  else
    hipLaunchKernelGGL(k_split_rows, dim3((unsigned)nq), dim3(256), 0, st, dq, nq, m, mp, Qh, Ql, qn, qr);
  prof_end(tok, st, 0.0);
  tok = prof_begin(PROF_NAIVE_GEMM, st);
  auto scan = [&](int64_t tiles, bool screen) {
    if (l1 && screen)
      hipLaunchKernelGGL((k_naive_f32<KNN_METRIC_L1, true>), dim3((unsigned)nranges, (unsigned)qt), dim3(256), 0, st,
                         Qh, nullptr, nullptr, nullptr, reinterpret_cast<const uint16_t *>(db->xpad), nullptr, nullptr,
                         nullptr, nq, n, mp, k, prange, c1, c2, part, candl, ncand, nranges, gtau, tiles);
    else if (screen)
      hipLaunchKernelGGL((k_naive_f32<KNN_METRIC_L2, true>), dim3((unsigned)nranges, (unsigned)qt), dim3(256), 0, st,
                         Qh, Ql, qn, qr, db->xbf, db->xbf + cells, db->norm_f, db->rownorm, nq, n, mp, k, prange, c1,
                         c2, part, candl, ncand, nranges, gtau, tiles);
    else if (l1)
      hipLaunchKernelGGL((k_naive_f32<KNN_METRIC_L1, false>), dim3((unsigned)nranges, (unsigned)qt), dim3(256), 0, st, Qh,
                         nullptr, nullptr, nullptr, reinterpret_cast<const uint16_t *>(db->xpad), nullptr, nullptr,
                         nullptr, nq, n, mp, k, prange, c1, c2, part, candl, ncand, nranges, gtau, tiles);
    else
      hipLaunchKernelGGL((k_naive_f32<KNN_METRIC_L2, false>), dim3((unsigned)nranges, (unsigned)qt), dim3(256), 0, st, Qh, Ql,
                         qn, qr, db->xbf, db->xbf + cells, db->norm_f, db->rownorm, nq, n, mp, k, prange, c1, c2, part,
                         candl, ncand, nranges, gtau, tiles);
  };
  // A probe over the first tiles of every range (the lists pass) gives
  // each query tau0, the k-th smallest upper bound of the union of the
  // ranges' lists: the upper bound of a real point, so tau0 >= d_(k), and
  // every true k-NN point has l <= d <= d_(k) <= tau0.  The full scan then
  // only screens: the pairs with l <= tau0 are the candidates, at least k
  // of them (the points that gave tau0).  Over a probe of s of the n
  // points about k n / s points lie below tau0, so s is sized for about
  // 1,024 candidates per query at most (the merge holds FCAP) and about
  // FCL / 4 per (query, range).
  const int64_t s_want = std::max<int64_t>(FPROBE_PTS, std::max<int64_t>((int64_t)k * n / 1024,
                                                                           (int64_t)k * n / (FCL / 4 * nranges)));
  const int64_t probe_tiles = std::max<int64_t>(FPROBE, (std::min(s_want, n) + nranges * FBP - 1) / (nranges * FBP));
  scan(probe_tiles, false);
  hipLaunchKernelGGL(k_naive_f32_tau0, dim3((unsigned)nq), dim3(256), 0, st, part, nranges, k, gtau);
  scan(INT64_MAX / 2 / FBP, true);
  // work units: l2 three BF16 products of 2 operations; l1 a difference and an addition
  prof_end(tok, st, (l1 ? 2.0 : 3.0 * 2.0) * (double)nq * (double)n * (double)m);
  tok = prof_begin(PROF_NAIVE_REST, st);
  hipLaunchKernelGGL(k_naive_f32_merge, dim3((unsigned)nq), dim3(FMT), 0, st, candl, ncand, nranges, k,
                     (const float *)db->X, dq, m, db->metric, out_idx, out_dist, flag, gtau);
  prof_end(tok, st, 0.0);
  HIP_TRY(hipGetLastError());
  // queries whose candidate list may be incomplete are rescanned exactly
  std::vector<int32_t> hflag(nq);
  HIP_TRY(hipMemcpyAsync(hflag.data(), flag, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<int32_t> redo;
  for (int64_t q = 0; q < nq; ++q)
    if (hflag[q]) redo.push_back((int32_t)q);
  prof_add_host(0, (uint64_t)redo.size());
  {
    const int rc = exact_f32_queries(db, dq, redo, k, out_idx, out_dist, st);
    if (rc != KNN_OK) return rc;
  }
  HIP_TRY(hipFreeAsync(ws, st));
  return KNN_OK;
}

}  // namespace knn
