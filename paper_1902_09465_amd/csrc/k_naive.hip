// k_naive.hip -- the naive scan of Section 3 (all distances, keep the k
// smallest) as a dense contraction on the gfx950 matrix cores.
//
// u8: with x' = x - 128 and q' = q - 128 (int8),
//       ||x - q||^2 = ||x'||^2 + ||q'||^2 - 2 x'.q',
//     x'.q' by v_mfma_i32_16x16x64_i8 (exact int32 for m <= 65536), so
//     distances are exact integers.  The k smallest (distance, index) per
//     query and point range are kept in registers or LDS while the tile
//     loop streams the points (fused epilogue, the n-by-nq distance matrix
//     is never stored); a merge takes the k smallest over the ranges.  For
//     k <= 64 the wide tile (128 queries x 256 points, stages loaded
//     straight into LDS) runs; l1 and larger k the 64 x 128 tile.
// f32: split-BF16 MFMA with an error bound and FP64 rescoring (k_naive_f32.hip).
// l1 distance (sum_j |x_j - q_j|; no product form, so no matrix cores): the
//     same tiles and top-k epilogue, with the tile's distances summed by
//     v_sad_u8 (four absolute differences and their sum per instruction) from
//     zero-padded u8 rows; exact in integers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "block_select.h"
#include "knn_host.h"
#include "knn_prof.h"

namespace knn {

typedef int v4i __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- DB prep

// u8: int8 copy x - 128 padded with zeros to mp (multiple of 64), and
// per-row sum of (x - 128)^2.
__global__ __launch_bounds__(256) void k_prep_u8_rows(const uint8_t *__restrict__ X, int64_t n, int64_t m,
                                                      int64_t mp, int8_t *__restrict__ xs, int32_t *__restrict__ nrm) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  int acc = 0;
  for (int64_t j = threadIdx.x; j < mp; j += 256) {
    int v = 0;
    if (j < m) v = (int)X[i * m + j] - 128;
    xs[i * mp + j] = (int8_t)v;
    acc += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ int red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) nrm[i] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_minmax_f32(const float *__restrict__ X, int64_t count, float *out) {
  float lo = INFINITY, hi = -INFINITY;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < count; p += (int64_t)gridDim.x * 256) {
    lo = fminf(lo, X[p]);
    hi = fmaxf(hi, X[p]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o));
    hi = fmaxf(hi, __shfl_xor(hi, o));
  }
  __shared__ float sl[4], sh[4];
  if ((threadIdx.x & 63) == 0) {
    sl[threadIdx.x >> 6] = lo;
    sh[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = fminf(fminf(sl[0], sl[1]), fminf(sl[2], sl[3]));
    out[2 * blockIdx.x + 1] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
  }
}

int db_range_f32(const float *X, int64_t count, double *lo, double *hi, hipStream_t st) {
  const int nb = 1024;
  float *d = nullptr;
  HIP_TRY(hipMalloc(&d, sizeof(float) * 2 * nb));
  hipLaunchKernelGGL(k_minmax_f32, dim3(nb), dim3(256), 0, st, X, count, d);
  std::vector<float> h(2 * nb);
  hipError_t e = hipMemcpy(h.data(), d, sizeof(float) * 2 * nb, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(KNN_EDEVICE, std::string("range: ") + hipGetErrorString(e));
  float l = INFINITY, u = -INFINITY;
  for (int b = 0; b < nb; ++b) {
    l = std::min(l, h[2 * b]);
    u = std::max(u, h[2 * b + 1]);
  }
  *lo = (double)l;
  *hi = (double)u;
  return KNN_OK;
}

// l1: rows copied with zero padding to mp elements (elem bytes each); the
// padding adds |0 - 0| = 0 to every distance.
__global__ __launch_bounds__(256) void k_pad_rows(const uint8_t *__restrict__ X, int64_t rows, int64_t m,
                                                  int64_t mp, int elem, uint8_t *__restrict__ out) {
  const int64_t r = blockIdx.x;
  if (r >= rows) return;
  const int64_t rb = m * elem, pb = mp * elem;
  for (int64_t b = threadIdx.x; b < pb; b += 256) out[r * pb + b] = b < rb ? X[r * rb + b] : (uint8_t)0;
}

void launch_pad_rows(const uint8_t *X, int64_t rows, int64_t m, int64_t mp, int elem, uint8_t *out, hipStream_t st) {
  hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)rows), dim3(256), 0, st, X, rows, m, mp, elem, out);
}

int naive_prepare_db(knn_db_s *db, hipStream_t st) {
  db->mp = (db->m + 63) / 64 * 64;
  if (db->metric == KNN_METRIC_L1) {
    const int elem = db->dtype == KNN_U8 ? 1 : 4;
    HIP_TRY(hipMalloc(&db->xpad, (size_t)db->n * db->mp * elem));
    hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)db->n), dim3(256), 0, st, db->X, db->n, db->m, db->mp, elem,
                       (uint8_t *)db->xpad);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return KNN_OK;
  }
  if (db->dtype == KNN_U8) {
    HIP_TRY(hipMalloc(&db->xs8, (size_t)db->n * db->mp));
    // norms padded to whole 256-point tiles (the wide scan loads a tile's
    // norms as one 1 KB piece)
    const size_t nn = (size_t)(db->n + 255) / 256 * 256;
    HIP_TRY(hipMalloc(&db->norm_i, sizeof(int32_t) * nn));
    HIP_TRY(hipMemsetAsync(db->norm_i, 0, sizeof(int32_t) * nn, st));
    hipLaunchKernelGGL(k_prep_u8_rows, dim3((unsigned)db->n), dim3(256), 0, st, db->X, db->n, db->m, db->mp,
                       db->xs8, db->norm_i);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return KNN_OK;
  }
  return naive_prepare_db_f32(db, st);
}

void naive_free_db(knn_db_s *db) {
  if (db->xs8) (void)hipFree(db->xs8);
  if (db->norm_i) (void)hipFree(db->norm_i);
  if (db->xbf) (void)hipFree(db->xbf);
  if (db->norm_f) (void)hipFree(db->norm_f);
  if (db->rownorm) (void)hipFree(db->rownorm);
  if (db->xpad) (void)hipFree(db->xpad);
  db->xpad = nullptr;
  db->xs8 = nullptr;
  db->norm_i = nullptr;
  db->xbf = nullptr;
  db->norm_f = nullptr;
  db->rownorm = nullptr;
}

// ---------------------------------------------------------------- u8 queries

__global__ __launch_bounds__(256) void k_prep_u8_queries(const uint8_t *__restrict__ Q, int64_t m, int64_t mp,
                                                         int8_t *__restrict__ qs, int32_t *__restrict__ qn) {
  const int64_t q = blockIdx.x;
  int acc = 0;
  for (int64_t j = threadIdx.x; j < mp; j += 256) {
    int v = 0;
    if (j < m) v = (int)Q[q * m + j] - 128;
    qs[q * mp + j] = (int8_t)v;
    acc += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ int red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) qn[q] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------- u8 scan

constexpr int NBQ = 64;    // queries per block tile
constexpr int NBP = 128;   // points per block tile
constexpr int DSTR = NBP + 4;  // row stride (4-byte words) of a tile's distances in LDS


// Distance of one tile entry: |q'|^2 + |x'|^2 - 2 x'.q' (squared l2; below
// 2^32 for m <= 65536) or the l1 sum itself.
template <int MET>
__device__ __forceinline__ uint32_t tile_dist(const int32_t *qn, const int32_t *xn, int64_t q, int64_t p, int acc) {
  if constexpr (MET == KNN_METRIC_L1) return (uint32_t)acc;
  return (uint32_t)((int64_t)qn[q] + (int64_t)xn[p] - 2 * (int64_t)acc);
}

// A pipeline slice is BK bytes of K (a multiple of the 64-byte MFMA step)
// of a tile of nbq query rows and NBP point rows; its LDS rows are padded by
// 16 bytes (conflict-free fragment reads).
constexpr int stage_bytes(int BK, int nbq = NBQ) { return (nbq + NBP) * (BK + 16); }
constexpr int BK_NAIVE = 128, BK_EXACT = 64;  // the scan's and the exact round's slices
// the exact round's query fragments per wave (block tile: 32 WA queries).
// Two for both distances: a 64 x 64 wave tile (four) doubles the fragment
// reuse but measured slower for squared l2 (1.07 vs 0.89 ms per round at
// 1024 x 100,000 x 3072: more registers, fewer waves), and the l1 tile
// would hold the query bytes of every fragment in registers.
template <int MET>
constexpr int exact_wa() { return 2; }
constexpr int CB = 32;                  // candidate buffer per query (<= 64)

// One block's 64 x 128 tile (queries q0.., points p0..) over the whole K
// range: x'.q' on the matrix cores (MET = squared l2, shifted int8 rows), or
// the l1 distance sum_j |x_j - q_j| by v_sad_u8 (MET = l1, zero-padded u8
// rows).  Either way lane l of wave w = 2 wq + wp ends with the value of
// query 32 wq + 16 a + 4 (l / 16) + v and point 64 wp + 16 b + l % 16 in
// acc[a][b][v] (the MFMA output layout).  The K loop runs over BK-byte
// slices through two LDS buffers (one barrier per slice); the global loads
// of the next PF slices are in flight in registers while the current slice
// is consumed, so each load has PF slices of compute to arrive.  Rows beyond
// nq / pend read as zeros.  smem: 2 x stage_bytes(BK) bytes.
//
// The K range is [kb, ke) of rows of mp bytes (kb and ke multiples of 64;
// the whole row by default).  With MASK, only the 4-byte words whose columns
// lie in [mlo, mhi) (multiples of 4) count: the others of the query rows
// are read as zeros (and, for l1, of the point rows too).
template <int MET, int PF, int BK, int WA = 2, bool MASK = false>
__device__ __forceinline__ void gemm_u8_tile(const int8_t *__restrict__ Q8, int64_t nq, const int8_t *__restrict__ X8,
                                             int64_t q0, int64_t p0, int64_t pr1, int64_t mp, uint8_t *smem,
                                             v4i (&acc)[WA][4], int64_t kb = 0, int64_t ke = -1, int64_t mlo = 0,
                                             int64_t mhi = 0) {
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int wq = wave >> 1, wp = wave & 1;
  constexpr int TQ = 32 * WA;  // query rows of the block tile (16 WA per wave)
  constexpr int BROW = BK + 16, STAGE = stage_bytes(BK, TQ);
  if (ke < 0) ke = mp;
  const int nks = (int)((ke - kb) / BK), tail = (int)((ke - kb) % BK);  // multiples of 64: tail 0 or 64 (BK 128)
  auto mask = [&](int64_t col, v4i &v) {
    if constexpr (MASK) {
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (col + 4 * d < mlo || col + 4 * d >= mhi) v[d] = 0;
    }
  };
#pragma unroll
  for (int a = 0; a < WA; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};
  // slice s covers K bytes [s BK, s BK + width): A TQ x width, B 128 x width
  // a slice is CPR 16-byte pieces per row: the 256 threads take NA pieces
  // of the query tile and NB of the point tile each
  constexpr int CPR = BK / 16, NA = TQ * CPR / 256, NB = NBP * CPR / 256;
  static_assert(NA * 256 == TQ * CPR && NB * 256 == NBP * CPR, "whole pieces per thread");
  auto load = [&](int64_t k0, int width, v4i (&ra)[NA], v4i (&rb)[NB]) {
    const int per_row = width / 16;
#pragma unroll
    for (int h = 0; h < NA; ++h) {
      const int e = tid + 256 * h, r = e / CPR, c = (e % CPR) * 16;
      ra[h] = v4i{0, 0, 0, 0};
      if (c / 16 < per_row && q0 + r < nq) ra[h] = *reinterpret_cast<const v4i *>(Q8 + (q0 + r) * mp + k0 + c);
      mask(k0 + c, ra[h]);
    }
#pragma unroll
    for (int h = 0; h < NB; ++h) {
      const int e = tid + 256 * h, r = e / CPR, c = (e % CPR) * 16;
      rb[h] = v4i{0, 0, 0, 0};
      if (c / 16 < per_row && p0 + r < pr1) rb[h] = *reinterpret_cast<const v4i *>(X8 + (p0 + r) * mp + k0 + c);
      if constexpr (MET == KNN_METRIC_L1) mask(k0 + c, rb[h]);
    }
  };
  auto store = [&](int buf, const v4i (&ra)[NA], const v4i (&rb)[NB]) {
    int8_t *As = reinterpret_cast<int8_t *>(smem) + buf * STAGE;
    int8_t *Bs = As + TQ * BROW;
#pragma unroll
    for (int h = 0; h < NA; ++h) {
      const int e = tid + 256 * h, r = e / CPR, c = (e % CPR) * 16;
      *reinterpret_cast<v4i *>(As + r * BROW + c) = ra[h];
    }
#pragma unroll
    for (int h = 0; h < NB; ++h) {
      const int e = tid + 256 * h, r = e / CPR, c = (e % CPR) * 16;
      *reinterpret_cast<v4i *>(Bs + r * BROW + c) = rb[h];
    }
  };
  auto compute = [&](int buf, int width) {
    const int8_t *As = reinterpret_cast<const int8_t *>(smem) + buf * STAGE;
    const int8_t *Bs = As + TQ * BROW;
    if constexpr (MET == KNN_METRIC_L1) {
      // 16 bytes of K at a time: the lane's 8 query rows and 4 point rows,
      // then 8 x 4 x 4 sums of absolute differences
      for (int kk = 0; kk < width; kk += 16) {
        v4i qv[WA][4], pv[4];
#pragma unroll
        for (int a = 0; a < WA; ++a)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            qv[a][v] = *reinterpret_cast<const v4i *>(As + (16 * WA * wq + 16 * a + 4 * (lane >> 4) + v) * BROW + kk);
#pragma unroll
        for (int b = 0; b < 4; ++b)
          pv[b] = *reinterpret_cast<const v4i *>(Bs + (64 * wp + 16 * b + (lane & 15)) * BROW + kk);
#pragma unroll
        for (int a = 0; a < WA; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              uint32_t t = (uint32_t)acc[a][b][v];
#pragma unroll
              for (int e = 0; e < 4; ++e) t = __builtin_amdgcn_sad_u8((uint32_t)qv[a][v][e], (uint32_t)pv[b][e], t);
              acc[a][b][v] = (int)t;
            }
      }
      return;
    }
    for (int kk = 0; kk < width; kk += 64) {
      v4i af[WA], bf[4];
#pragma unroll
      for (int a = 0; a < WA; ++a)
        af[a] = *reinterpret_cast<const v4i *>(As + (16 * WA * wq + 16 * a + (lane & 15)) * BROW + kk + 16 * (lane >> 4));
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bf[b] = *reinterpret_cast<const v4i *>(Bs + (64 * wp + 16 * b + (lane & 15)) * BROW + kk + 16 * (lane >> 4));
#pragma unroll
      for (int a = 0; a < WA; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  };
  static_assert(BK % 64 == 0, "whole MFMA K steps per slice");
  const int nsl = nks + (tail ? 1 : 0);
  auto width = [&](int s) { return s < nks ? BK : tail; };
  // PF register stages: stage u holds slices u, u + PF, ...; a stage is
  // refilled once its slice is in LDS, PF slices before it is stored again
  constexpr int NS = PF;
  v4i ra[NS][NA], rb[NS][NB];
#pragma unroll
  for (int u = 0; u < NS; ++u)
    if (u < nsl) load(kb + (int64_t)u * BK, width(u), ra[u], rb[u]);
  store(0, ra[0], rb[0]);
  __syncthreads();
  for (int base = 0; base < nsl; base += NS) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int sl = base + u;
      if (sl >= nsl) break;
      // stage u was stored to LDS in the previous iteration: refill it
      if (sl + NS < nsl) load(kb + (int64_t)(sl + NS) * BK, width(sl + NS), ra[u], rb[u]);
      compute(sl & 1, width(sl));
      if (sl + 1 < nsl) store((sl + 1) & 1, ra[(u + 1) % NS], rb[(u + 1) % NS]);
      __syncthreads();
    }
  }
}

// The scan for k <= 64:
//  * the K loop is double-buffered: the next BK-byte slice of the query
//    and point tiles is loaded into registers while the current one is
//    consumed from LDS (one barrier per slice);
//  * the per-query k smallest live in registers, one sorted list per query
//    spread over the lanes of the wave that owns it (lane j holds the j-th
//    smallest).  A tile's distances are filtered against the list's k-th
//    key and the few that pass are appended to a per-query LDS buffer; the
//    buffer is merged into the list by a wave sort when it would overflow
//    and at the end of the block (sort, reverse, take the smaller of each
//    pair, bitonic clean-up: the 64 smallest of both, sorted).
template <int MET>
__global__ __launch_bounds__(256) void k_naive_u8_k64(const int8_t *__restrict__ Q8, const int32_t *__restrict__ qn,
                                                      const int8_t *__restrict__ X8, const int32_t *__restrict__ xn,
                                                      int64_t nq, int64_t n, int64_t mp, int k, int64_t prange,
                                                      uint64_t *__restrict__ part, int64_t nranges) {
  constexpr uint64_t PAD = ~0ull;
  constexpr int QPW = NBQ / 4;  // queries owned by one wave in the epilogue
  __shared__ __align__(16) uint8_t smem[2 * stage_bytes(BK_NAIVE) > NBQ * DSTR * 4 ? 2 * stage_bytes(BK_NAIVE)
                                                                                     : NBQ * DSTR * 4];
  __shared__ uint64_t Cb[NBQ][CB];
  uint32_t *Ds = reinterpret_cast<uint32_t *>(smem);
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int64_t q0 = (int64_t)blockIdx.y * NBQ;
  const int64_t pr0 = (int64_t)blockIdx.x * prange;
  const int64_t pr1 = std::min(n, pr0 + prange);
  const int wq = wave >> 1, wp = wave & 1;
  uint64_t L[QPW];   // lane j: j-th smallest of query wave*QPW + t (its k-th, read from lane k - 1,
                     // is the filter threshold; PAD while fewer than k)
  int cnt[QPW];      // keys in the query's buffer
#pragma unroll
  for (int t = 0; t < QPW; ++t) {
    L[t] = PAD;
    cnt[t] = 0;
  }
  for (int64_t p0 = pr0; p0 < pr1; p0 += NBP) {
    v4i acc[2][4];
    gemm_u8_tile<MET, 1, BK_NAIVE>(Q8, nq, X8, q0, p0, pr1, mp, smem, acc);
    // distances of the tile into LDS (the stage buffers are free now)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ql = 32 * wq + 16 * a + 4 * (lane >> 4) + v;
          const int pl = 64 * wp + 16 * b + (lane & 15);
          uint32_t d = 0xFFFFFFFFu;
          if (p0 + pl < pr1 && q0 + ql < nq) d = tile_dist<MET>(qn, xn, q0 + ql, p0 + pl, acc[a][b][v]);
          Ds[ql * DSTR + pl] = d;
        }
    __syncthreads();
    // filter against the k-th key, append to the buffer, merge when full
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
#pragma unroll
    for (int t = 0; t < QPW; ++t) {
      const int ql = wave * QPW + t;
      const uint32_t d0 = Ds[ql * DSTR + lane], d1 = Ds[ql * DSTR + lane + 64];
      const uint64_t c0 = d0 == 0xFFFFFFFFu ? PAD : (((uint64_t)d0 << 32) | (uint64_t)(p0 + lane));
      const uint64_t c1 = d1 == 0xFFFFFFFFu ? PAD : (((uint64_t)d1 << 32) | (uint64_t)(p0 + lane + 64));
      const uint64_t tau = wave_bcast_u64(L[t], k - 1);
      const bool a0 = c0 < tau, a1 = c1 < tau;
      const uint64_t m0 = __ballot(a0), m1 = __ballot(a1);
      if ((m0 | m1) == 0) continue;  // wave-uniform
      const int n0 = __popcll(m0), n1 = __popcll(m1);
      if (cnt[t] + n0 + n1 > CB) {
        // does not fit: merge the buffer (written in earlier tiles, before
        // the last barrier) and this tile's candidates into the list
        if (cnt[t] > 0) L[t] = merge_sorted64(L[t], lane < cnt[t] ? Cb[ql][lane] : PAD);
        L[t] = merge_sorted64(L[t], a0 ? c0 : PAD);
        L[t] = merge_sorted64(L[t], a1 ? c1 : PAD);
        cnt[t] = 0;
        continue;
      }
      if (a0) Cb[ql][cnt[t] + __popcll(m0 & lt)] = c0;
      if (a1) Cb[ql][cnt[t] + n0 + __popcll(m1 & lt)] = c1;
      cnt[t] += n0 + n1;
    }
    __syncthreads();
  }
  // final merge and the block's k smallest per query -> part[q][range][k]
#pragma unroll
  for (int t = 0; t < QPW; ++t) {
    const int ql = wave * QPW + t;  // its buffer was written before the last barrier
    if (cnt[t] > 0) L[t] = merge_sorted64(L[t], lane < cnt[t] ? Cb[ql][lane] : PAD);
    if (q0 + ql < nq && lane < k) part[((q0 + ql) * nranges + blockIdx.x) * (int64_t)k + lane] = L[t];
  }
}

// The scan for 64 < k <= KC: per-query sorted lists of KC keys in LDS,
// filled by topk_insert from each tile's distances.
template <int KC, int MET>
__global__ __launch_bounds__(256) void k_naive_u8(const int8_t *__restrict__ Q8, const int32_t *__restrict__ qn,
                                                  const int8_t *__restrict__ X8, const int32_t *__restrict__ xn,
                                                  int64_t nq, int64_t n, int64_t mp, int k, int64_t prange,
                                                  uint64_t *__restrict__ part, int64_t nranges) {
  // the pipeline stages and the distance tile are never live at the same time
  __shared__ __align__(16) uint8_t smem[2 * stage_bytes(BK_NAIVE) > NBQ * DSTR * 4 ? 2 * stage_bytes(BK_NAIVE)
                                                                                     : NBQ * DSTR * 4];
  uint32_t *Ds = reinterpret_cast<uint32_t *>(smem);
  __shared__ uint64_t L[NBQ * KC];
  __shared__ uint64_t Tau[NBQ];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int64_t q0 = (int64_t)blockIdx.y * NBQ;
  const int64_t pr0 = (int64_t)blockIdx.x * prange;
  const int64_t pr1 = std::min(n, pr0 + prange);
  // sentinel list entries: unique keys above every real key
  for (int j = tid; j < NBQ * KC; j += 256) L[j] = ~0ull - (uint64_t)(j % KC);
  const int wq = wave >> 1, wp = wave & 1;
  for (int j = tid; j < NBQ; j += 256) Tau[j] = ~0ull;
  __syncthreads();
  for (int64_t p0 = pr0; p0 < pr1; p0 += NBP) {
    v4i acc[2][4];
    gemm_u8_tile<MET, 1, BK_NAIVE>(Q8, nq, X8, q0, p0, pr1, mp, smem, acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ql = 32 * wq + 16 * a + 4 * (lane >> 4) + v;
          const int pl = 64 * wp + 16 * b + (lane & 15);
          uint32_t d = 0xFFFFFFFFu;
          if (p0 + pl < pr1 && q0 + ql < nq) d = tile_dist<MET>(qn, xn, q0 + ql, p0 + pl, acc[a][b][v]);
          Ds[ql * DSTR + pl] = d;
        }
    __syncthreads();
    // per-query top-k, wave `wave` owns queries [16 wave, 16 wave + 16)
#pragma unroll 1
    for (int t = 0; t < NBQ / 4; ++t) {
      const int ql = wave * (NBQ / 4) + t;
      if (q0 + ql >= nq) break;
      const uint32_t d0 = Ds[ql * DSTR + lane], d1 = Ds[ql * DSTR + lane + 64];
      const uint64_t c0 = d0 == 0xFFFFFFFFu ? ~0ull : (((uint64_t)d0 << 32) | (uint64_t)(p0 + lane));
      const uint64_t c1 = d1 == 0xFFFFFFFFu ? ~0ull : (((uint64_t)d1 << 32) | (uint64_t)(p0 + lane + 64));
      uint64_t tau = Tau[ql];
      topk_insert<KC>(L + ql * KC, k, tau, c0, c1);
      if (lane == 0) Tau[ql] = tau;
    }
    __syncthreads();
  }
  // the block's k smallest per query -> part[q][range][k]
  for (int t = 0; t < NBQ / 4; ++t) {
    const int ql = wave * (NBQ / 4) + t;
    if (q0 + ql >= nq) break;
    uint64_t *dst = part + ((q0 + ql) * nranges + blockIdx.x) * (int64_t)k;
    for (int j = lane; j < k; j += 64) dst[j] = L[ql * KC + j];
  }
}

// ---------------------------------------------------------------- exact round, query-lane batches

// Shifted int8 copies of the running slots' queries, padded to mp, and their
// squared norms (zero rows for idle slots): the A operand of the exact round.
// For the l1 distance the rows are the queries' own bytes, zero-padded.
template <int MET>
__global__ __launch_bounds__(256) void k_build_q8(const Slot *__restrict__ slots, int32_t ns, int64_t m, int64_t mp,
                                                  int8_t *__restrict__ Q8, int32_t *__restrict__ qn) {
  const int s = blockIdx.x;
  const bool run = s < ns && slots[s].state == 1;
  const uint8_t *q = run ? reinterpret_cast<const uint8_t *>(slots[s].q) : nullptr;
  if constexpr (MET == KNN_METRIC_L1) {
    for (int64_t j = threadIdx.x; j < mp; j += 256)
      reinterpret_cast<uint8_t *>(Q8)[(int64_t)s * mp + j] = (run && j < m) ? q[j] : (uint8_t)0;
    return;
  }
  int acc = 0;
  for (int64_t j = threadIdx.x; j < mp; j += 256) {
    const int v = (run && j < m) ? (int)q[j] - 128 : 0;
    Q8[(int64_t)s * mp + j] = (int8_t)v;
    acc += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ int red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) qn[s] = red[0] + red[1] + red[2] + red[3];
}

// The exact round of a batch whose slots all run it together, as one GEMM
// over (slots x points): S = |q'|^2 + |x'|^2 - 2 q'.x' for every undecided
// sampled pair (flag 0; every pair when the round is round 0), flag exact.
// Exact in integers (int8 MFMA, int32 accumulation, m <= 65536).  For the l1
// distance the same tiles sum |x_j - q_j| with v_sad_u8 on zero-padded rows.
template <int MET, int PF>
__global__ __launch_bounds__(256) void k_exact_ql_u8(const Slot *__restrict__ slots, const int8_t *__restrict__ Q8,
                                                     const int32_t *__restrict__ qn, const int8_t *__restrict__ X8,
                                                     const int32_t *__restrict__ xn, Bufs B, Geometry G, int32_t cur,
                                                     int32_t impl, uint32_t *__restrict__ Dpm, int32_t nqp) {
  // block tile XQ queries x NBP points: each wave 16 XWA queries x 64 points
  constexpr int XWA = exact_wa<MET>(), XQ = 32 * XWA;
  // the K loop's stages, then the tile's point-major sums for the stores
  constexpr int TROW = XQ + 4;  // words per point row of the staged sums (16-byte aligned rows)
  constexpr int SMEM = 2 * stage_bytes(BK_EXACT, XQ) > NBP * TROW * 4 ? 2 * stage_bytes(BK_EXACT, XQ)
                                                                       : NBP * TROW * 4;
  __shared__ __align__(16) uint8_t smem[SMEM];
  const int64_t n = G.n, mp = G.mp;
  const int ns = G.nslots;
  // work item (point tile, query tile), query tile fastest: the query tiles
  // of one point tile read the same point rows, so they run back to back on
  // one XCD and the rows come from its L2
  const int64_t nqt = (ns + XQ - 1) / XQ, nwork = nqt * ((n + NBP - 1) / NBP);
  const int64_t w = xcd_work_item(nwork);
  if (w >= nwork) return;
  const int64_t p0 = (w / nqt) * NBP;
  const int64_t q0 = (w % nqt) * XQ;
  const int64_t pend = std::min(n, p0 + NBP);
  // which of the tile's slots take this pass (read once, before the K loop)
  __shared__ uint8_t take[XQ];
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (threadIdx.x < XQ) {
    const int64_t s = q0 + threadIdx.x;
    bool t = s < ns && slots[s].state == 1 && slots[s].cur == cur;
    if (t && G.flagsets && slots[s].implicit == 0) t = false;  // a sparse slot: its own exact pass
    take[threadIdx.x] = t ? 1 : 0;
    if (t) any = 1;
  }
  __syncthreads();
  if (!any) return;  // (block-uniform) no slot of this query tile takes the pass
  v4i acc[XWA][4];
  gemm_u8_tile<MET, PF, BK_EXACT, XWA>(Q8, (int64_t)ns, X8, q0, p0, pend, mp, smem, acc);  // (its barriers publish take[])
  const int lane = lane_id(), wave = threadIdx.x >> 6, wq = wave >> 1, wp = wave & 1;
  uint64_t my_pairs = 0;
  // point-major batches: the sums go through LDS as [point][query] rows, so
  // that each point's queries are stored as 16-byte pieces (a pair that
  // keeps its sum is marked ~0, above every sum: m * 65025 < 2^32 - 1)
  uint32_t *T = reinterpret_cast<uint32_t *>(smem);  // (the K loop ended with a barrier)
#pragma unroll
  for (int a = 0; a < XWA; ++a) {
    // this fragment row's flags first, all loads in flight together (flag
    // 0: an undecided sampled pair, the only ones made exact; every pair in
    // round 0)
    uint8_t fv[4][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ql = 16 * XWA * wq + 16 * a + 4 * (lane >> 4) + v;
      const int64_t s = q0 + ql;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t i = p0 + 64 * wp + 16 * b + (lane & 15);
        fv[v][b] = (take[ql] && i < n) ? (impl ? (uint8_t)0 : B.fl[s * n + i]) : (uint8_t)1;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ql = 16 * XWA * wq + 16 * a + 4 * (lane >> 4) + v;
      const int64_t s = q0 + ql;
      const int64_t qs = (MET == KNN_METRIC_L1 || s >= ns) ? 0 : qn[s];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int pl = 64 * wp + 16 * b + (lane & 15);
        if (fv[v][b] != 0) {
          if (G.flagsets) T[pl * TROW + ql] = ~0u;
          continue;
        }
        const int64_t i = p0 + pl;
        const int64_t off = s * n + i;
        const int64_t v64 = MET == KNN_METRIC_L1 ? (int64_t)(uint32_t)acc[a][b][v]
                                                 : qs + (int64_t)xn[i] - 2 * (int64_t)acc[a][b][v];
        if (G.flagsets) {
          // point-major sums (below 2^32 for m <= 65536); the round of the
          // pair's last samples is recorded with its exact flag
          T[pl * TROW + ql] = (uint32_t)v64;
          B.ri[off] = impl ? (uint8_t)0 : (uint8_t)(cur - 1);
        } else {
          B.S[off] = v64;
          if (impl) B.ri[off] = 0;
        }
        B.fl[off] = FL_EXACT;
        ++my_pairs;
      }
    }
  }
  if (G.flagsets) {
    __syncthreads();
    // 16-byte pieces: NBP rows x XQ / 4 pieces (nqp is a multiple of 16, so
    // a piece's four queries are all below nqp or all at or past it)
    constexpr int PIECES = NBP * XQ / 4;
    for (int e = threadIdx.x; e < PIECES; e += 256) {
      const int pl = e / (XQ / 4), qc = 4 * (e % (XQ / 4));
      const int64_t i = p0 + pl, s = q0 + qc;
      if (i >= n || s >= nqp) continue;
      const uint4 val = *reinterpret_cast<const uint4 *>(&T[pl * TROW + qc]);
      uint32_t *dst = Dpm + i * nqp + s;
      if (val.x != ~0u && val.y != ~0u && val.z != ~0u && val.w != ~0u) {
        *reinterpret_cast<uint4 *>(dst) = val;
      } else {
        if (val.x != ~0u) dst[0] = val.x;
        if (val.y != ~0u) dst[1] = val.y;
        if (val.z != ~0u) dst[2] = val.z;
        if (val.w != ~0u) dst[3] = val.w;
      }
    }
  }
  if (G.prof) {  // whole waves reach this point
    wave_count_add(&prof_copy(G.prof)[0], my_pairs * (uint64_t)(G.m + 14));
    wave_count_add(&prof_copy(G.prof)[2], my_pairs * (uint64_t)G.m);
  }
}

// One round of a point-major batch whose queries share one coordinate
// sequence (sampling 2 or 3): the round's samples t0 <= t < t1 are columns
// [t0, t1) of the gathered copies QS [nqp][kp] and XS [n][kp], so the sums
// of all (query, point) pairs are one product over that column range, on
// the same tiles as the exact round.  For squared l2 a pair's round sum is
// |x'|^2 + |q'|^2 - 2 x'.q' over the range (x' = x - 128; the range norms are
// differences of the prefix norms at boundaries lo and hi); for l1 the
// v_sad_u8 sum over the range.  The sum is added to the pair's running sum
// in D where the pair is sampled this round (its "not sampled" byte in A is
// zero; round 0: every pair of a running slot, D starts from zero).  The
// exact round of sampling without replacement (exact = 1) adds the
// coordinates not seen yet, [T_{R-1}, m): the running sum becomes the exact
// distance, and the pair is marked exact as in k_exact_ql_u8.
template <int MET, int PF>
__global__ __launch_bounds__(256) void k_round_seq_u8(const Slot *__restrict__ slots, const int8_t *__restrict__ QS,
                                                      const int8_t *__restrict__ XS, int64_t kp,
                                                      const int32_t *__restrict__ qn, const int32_t *__restrict__ xn,
                                                      int32_t lo, int32_t hi, int64_t t0, int64_t t1,
                                                      const uint8_t *__restrict__ A, uint32_t *__restrict__ D,
                                                      int32_t nqp, Bufs B, Geometry G, int32_t cur, int32_t impl,
                                                      int32_t exact) {
  constexpr int XWA = exact_wa<MET>(), XQ = 32 * XWA;
  __shared__ __align__(16) uint8_t smem[2 * stage_bytes(BK_EXACT, XQ)];
  const int64_t n = G.n;
  const int ns = G.nslots;
  const int64_t nqt = (ns + XQ - 1) / XQ, nwork = nqt * ((n + NBP - 1) / NBP);
  const int64_t w = xcd_work_item(nwork);
  if (w >= nwork) return;
  const int64_t p0 = (w / nqt) * NBP;
  const int64_t q0 = (w % nqt) * XQ;
  const int64_t pend = std::min(n, p0 + NBP);
  __shared__ uint8_t take[XQ];
  const int lane = lane_id(), wave = threadIdx.x >> 6, wq = wave >> 1, wp = wave & 1;
  // the range norms |x'|^2 and |q'|^2 over [lo, hi) of the tile's points and
  // queries; they and the slots' flags load together, before the products
  __shared__ uint32_t xrl[NBP], qrl[XQ];
  bool tmine = false;
  if (threadIdx.x < XQ) {
    const int64_t s = q0 + threadIdx.x;
    tmine = s < ns && slots[s].state == 1 && slots[s].cur == cur && slots[s].implicit != 0;
    take[threadIdx.x] = tmine ? 1 : 0;
  }
  if (threadIdx.x < NBP) {
    const int64_t i = p0 + threadIdx.x;
    xrl[threadIdx.x] =
        (MET == KNN_METRIC_L2 && i < n) ? (uint32_t)(xn[(int64_t)hi * n + i] - xn[(int64_t)lo * n + i]) : 0u;
  } else if (threadIdx.x < NBP + XQ) {
    const int64_t s = q0 + threadIdx.x - NBP;
    qrl[threadIdx.x - NBP] =
        (MET == KNN_METRIC_L2 && s < nqp) ? (uint32_t)(qn[(int64_t)hi * nqp + s] - qn[(int64_t)lo * nqp + s]) : 0u;
  }
  if (!__syncthreads_or(tmine)) return;  // (block-uniform) no dense slot of this query tile runs this round
  // the K slices covering [t0, t1); words outside it count as zero
  const int64_t kb = t0 / 64 * 64, ke = std::min<int64_t>(kp, (t1 + 63) / 64 * 64);
  v4i acc[XWA][4];
  gemm_u8_tile<MET, PF, BK_EXACT, XWA, true>(QS, (int64_t)nqp, XS, q0, p0, pend, kp, smem, acc, kb, ke, t0, t1);
  uint64_t my_pairs = 0;
  if (exact && (n & 15) == 0 && p0 + NBP <= n) {
    // pairs made exact: the undecided sampled ones (flag 0).  A whole tile
    // with 16-byte aligned flag rows: each thread takes 32 consecutive
    // points of one query (four threads per row of the tile), reads their
    // flags and round bytes as 16-byte words, and rewrites the words that
    // hold a zero flag (flag FL_EXACT, round cur - 1; with implicit sets
    // every pair is undecided and nothing is read)
    static_assert(XQ * NBP == 256 * 32, "32 points of one query per thread");
    static_assert(FL_EXACT == 1, "a zero byte becomes FL_EXACT by or-ing in its bit 0");
    const int r = threadIdx.x >> 2;
    if (take[r]) {
      const int64_t off = (q0 + r) * n + p0 + 32 * (threadIdx.x & 3);
      const uint32_t rep = 0x01010101u * (impl ? 0u : (uint32_t)(uint8_t)(cur - 1));
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint4 fw = impl ? make_uint4(0u, 0u, 0u, 0u) : *reinterpret_cast<const uint4 *>(B.fl + off + 16 * h);
        const uint32_t fv[4] = {fw.x, fw.y, fw.z, fw.w};
        uint32_t zm[4], any = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {  // bit 7 of each zero byte
          zm[e] = ~((((fv[e] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | fv[e])) & 0x80808080u;
          any |= zm[e];
          my_pairs += (uint64_t)__popc(zm[e]);
        }
        if (any) {
          const uint4 rw = impl ? make_uint4(0u, 0u, 0u, 0u) : *reinterpret_cast<const uint4 *>(B.ri + off + 16 * h);
          const uint32_t rv[4] = {rw.x, rw.y, rw.z, rw.w};
          uint32_t nf[4], nr[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t mk = (zm[e] >> 7) * 0xFFu;  // 0xFF in each zero byte
            nf[e] = fv[e] | (zm[e] >> 7);            // FL_EXACT
            nr[e] = (rv[e] & ~mk) | (rep & mk);
          }
          *reinterpret_cast<uint4 *>(B.fl + off + 16 * h) = make_uint4(nf[0], nf[1], nf[2], nf[3]);
          *reinterpret_cast<uint4 *>(B.ri + off + 16 * h) = make_uint4(nr[0], nr[1], nr[2], nr[3]);
        }
      }
    }
  } else if (exact) {
    // (the last, partial tile, or flag rows not 16-byte aligned) marked in
    // the fragment layout (sixteen consecutive points of one query per lane
    // group), all flag loads of a fragment row in flight together
#pragma unroll
    for (int a = 0; a < XWA; ++a) {
      uint8_t fv[4][4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ql = 16 * XWA * wq + 16 * a + 4 * (lane >> 4) + v;
        const int64_t s = q0 + ql;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int64_t i = p0 + 64 * wp + 16 * b + (lane & 15);
          fv[v][b] = (take[ql] && i < n) ? (impl ? (uint8_t)0 : B.fl[s * n + i]) : (uint8_t)1;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t s = q0 + 16 * XWA * wq + 16 * a + 4 * (lane >> 4) + v;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if (fv[v][b] != 0) continue;
          const int64_t off = s * n + p0 + 64 * wp + 16 * b + (lane & 15);
          B.fl[off] = FL_EXACT;
          B.ri[off] = impl ? (uint8_t)0 : (uint8_t)(cur - 1);
          ++my_pairs;
        }
      }
    }
  }
  // The round sums go to D straight from the fragment layout: for query
  // group a and point group b a lane holds four consecutive queries of one
  // point, one 16-byte piece of that point's row of D (nqp is a multiple
  // of 16, so the four are all below nqp or all at or past it).  Per query
  // group the pieces' "not sampled" words and old sums of all four point
  // groups are loaded together, then added to and stored.  Sums are taken
  // mod 2^32: every running sum is below 2^32 (m <= 65536).
#pragma unroll
  for (int a = 0; a < XWA; ++a) {
    const int ql = 16 * XWA * wq + 16 * a + 4 * (lane >> 4);
    const int64_t s = q0 + ql;
    const uint32_t tk = take[ql] | (take[ql + 1] << 8) | (take[ql + 2] << 16) | (take[ql + 3] << 24);
    uint32_t xr[4], qr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xr[e] = xrl[64 * wp + 16 * e + (lane & 15)];
      qr[e] = qrl[ql + e];
    }
    uint32_t a4[4];
    uint4 old[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {  // all loads of the query group in flight together
      const int64_t i = p0 + 64 * wp + 16 * b + (lane & 15);
      const bool ok = i < n && s < nqp && tk != 0 && !impl;
      a4[b] = ok ? *reinterpret_cast<const uint32_t *>(A + i * nqp + s) : 0u;
      old[b] = ok ? *reinterpret_cast<const uint4 *>(D + i * nqp + s) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t i = p0 + 64 * wp + 16 * b + (lane & 15);
      if (i >= n || s >= nqp || tk == 0) continue;
      const uint32_t oo[4] = {old[b].x, old[b].y, old[b].z, old[b].w};
      uint32_t nw[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t val = MET == KNN_METRIC_L1 ? (uint32_t)acc[a][b][v]
                                                  : xr[b] + qr[v] - 2u * (uint32_t)acc[a][b][v];
        const bool sampled = ((tk >> (8 * v)) & 1u) != 0 && ((a4[b] >> (8 * v)) & 255u) == 0;
        nw[v] = sampled ? oo[v] + val : oo[v];
        if (sampled && !exact) ++my_pairs;
      }
      *reinterpret_cast<uint4 *>(D + i * nqp + s) = make_uint4(nw[0], nw[1], nw[2], nw[3]);
    }
  }
  if (G.prof) {  // whole waves reach this point
    wave_count_add(&prof_copy(G.prof)[exact ? 2 : 1], my_pairs * (uint64_t)(t1 - t0));
  }
}

void launch_round_seq_u8(const Slot *slots, const SeqBufs &q, int32_t lo, int32_t hi, int64_t t0, int64_t t1,
                         const uint8_t *A, uint32_t *D, int32_t nqp, const Bufs &B, const Geometry &G, int32_t cur,
                         int32_t impl, int32_t exact, hipStream_t st) {
  const int xq = 32 * (G.metric == KNN_METRIC_L1 ? exact_wa<KNN_METRIC_L1>() : exact_wa<KNN_METRIC_L2>());
  const int64_t nwork = ((G.n + NBP - 1) / NBP) * ((G.nslots + xq - 1) / xq);
  const dim3 grid((unsigned)xcd_grid(nwork));
  if (G.metric == KNN_METRIC_L1)
    hipLaunchKernelGGL((k_round_seq_u8<KNN_METRIC_L1, 3>), grid, dim3(256), 0, st, slots, q.qs, q.xs, q.kp, q.qn, q.xn,
                       lo, hi, t0, t1, A, D, nqp, B, G, cur, impl, exact);
  else
    hipLaunchKernelGGL((k_round_seq_u8<KNN_METRIC_L2, 3>), grid, dim3(256), 0, st, slots, q.qs, q.xs, q.kp, q.qn, q.xn,
                       lo, hi, t0, t1, A, D, nqp, B, G, cur, impl, exact);
}

void launch_build_q8(const Slot *slots, int32_t ns, int64_t m, int64_t mp, int8_t *Q8, int32_t *qn, int32_t metric,
                     hipStream_t st) {
  if (metric == KNN_METRIC_L1)
    hipLaunchKernelGGL(k_build_q8<KNN_METRIC_L1>, dim3((unsigned)ns), dim3(256), 0, st, slots, ns, m, mp, Q8, qn);
  else
    hipLaunchKernelGGL(k_build_q8<KNN_METRIC_L2>, dim3((unsigned)ns), dim3(256), 0, st, slots, ns, m, mp, Q8, qn);
}

void launch_exact_ql_u8(const Slot *slots, const int8_t *Q8, const int32_t *qn, const int8_t *X8, const int32_t *xn,
                        const Bufs &B, const Geometry &G, int32_t cur, int32_t impl, uint32_t *Dpm, int32_t nqp,
                        hipStream_t st) {
  const int xq = 32 * (G.metric == KNN_METRIC_L1 ? exact_wa<KNN_METRIC_L1>() : exact_wa<KNN_METRIC_L2>());
  const int64_t nwork = ((G.n + NBP - 1) / NBP) * ((G.nslots + xq - 1) / xq);
  const dim3 grid((unsigned)xcd_grid(nwork));
  // slices of global loads in flight per thread (KNN_EXACT_PF: 3 (default), 4 or 6)
  const int pf = [] {  // (read per launch, like the other knobs)
    const char *e = std::getenv("KNN_EXACT_PF");
    const int v = e ? std::atoi(e) : 3;
    return (v == 4 || v == 6) ? v : 3;
  }();
#define KNN_EXACT_LAUNCH(MET_, PF_)                                                                           \
  hipLaunchKernelGGL((k_exact_ql_u8<MET_, PF_>), grid, dim3(256), 0, st, slots, Q8, qn, X8, xn, B, G, cur, impl, \
                     Dpm, nqp)
  if (G.metric == KNN_METRIC_L1) {
    if (pf == 3) KNN_EXACT_LAUNCH(KNN_METRIC_L1, 3);
    else if (pf == 4) KNN_EXACT_LAUNCH(KNN_METRIC_L1, 4);
    else KNN_EXACT_LAUNCH(KNN_METRIC_L1, 6);
  } else {
    if (pf == 3) KNN_EXACT_LAUNCH(KNN_METRIC_L2, 3);
    else if (pf == 4) KNN_EXACT_LAUNCH(KNN_METRIC_L2, 4);
    else KNN_EXACT_LAUNCH(KNN_METRIC_L2, 6);
  }
#undef KNN_EXACT_LAUNCH
}

// ---------------------------------------------------------------- wide u8 scan (squared l2, k <= 64)

__global__ void k_fill_u64(uint64_t *p, uint64_t v) { p[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = v; }

// Block tile 128 queries x 256 points, eight waves of 64 x 64 (wave w:
// queries 64 (w >> 2) + [0, 64), points 64 (w & 3) + [0, 64); the MFMA
// output layout as in gemm_u8_tile).  The K loop runs over 64-byte stages of
// both row tiles held in a ring of NST LDS buffers.  Stages arrive by direct
// global-to-LDS loads (global_load_lds_dwordx4: one wave instruction moves
// 16 rows x 64 bytes, lane j writing bytes [16 j, 16 j + 16) of its 1 KB), so
// nothing is staged in registers.  A row's four 16-byte pieces are stored permuted by
// wswz(row), which makes the fragment reads (16 rows, one piece each)
// conflict-free.  A stage's fragments are read into registers while the
// previous stage's products run, so NST - 2 stages are in flight during the
// products.  The stage stream runs on across the block's tiles: the next
// tile's first stages load during a tile's epilogue.
namespace wide {
constexpr int TQ = 128, TP = 256, BK = 64;
constexpr int STAGE = (TQ + TP) * BK;           // 24 KB
constexpr int DMA = STAGE / 1024 / 8;           // wave instructions per wave and stage (3)
constexpr int SUB = 8;                          // candidates per (query, point quarter) and tile (< 0x77)
constexpr int WSTR = 68;                        // row stride (words) of a staged wave tile
// (measured: no LDS bank conflicts on gfx950 with this permutation; the
// fragment reads of a 64-byte-row layout without it conflict)
__device__ __forceinline__ int wswz(int r) { return (r >> 1) & 3; }
// s_waitcnt with only the vector-memory count bounded (expcnt and lgkmcnt at
// their maxima)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x70 | 0xF00);
}
}  // namespace wide

// One wave-wide global-to-LDS load: 16 bytes per lane from gptr to LDS bytes
// [lds + 16 lane, lds + 16 lane + 16) (lds the same in every lane).  Inline
// asm rather than the builtin: the compiler cannot tell the ring's buffers
// apart and would wait for every load in flight before each LDS read; the
// ring's own waits (wide_sync) order these writes before their reads.  No
// register is written (the data goes to LDS), so nothing is left pending in
// registers.
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
  return (uint32_t)(uintptr_t)((__attribute__((address_space(3))) const void *)p);
}
__device__ __forceinline__ void lds_load16(const void *gptr, uint32_t lds) {
  const uint32_t a = __builtin_amdgcn_readfirstlane(lds);
  uint32_t m0_saved;  // m0 is restored for the compiler's own uses
  asm volatile(
      "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off\n\ts_mov_b32 m0, %0"
      : "=&s"(m0_saved)
      : "v"(gptr), "s"(a)
      : "memory");
}

// The 16-byte piece of K this lane loads for every stage row it fills (row
// 16 e + lane / 4 of the stage's 1 KB piece e): (lane % 4) ^ wswz(row), where
// the row's low four bits are lane / 4.
__device__ __forceinline__ int wide_piece(int lane) { return 16 * ((lane & 3) ^ wide::wswz(lane >> 2)); }

// The wave's fragments of one stage (K step 64): query rows 64 wq + 16 a,
// point rows 64 wp + 16 b of the stage.
__device__ __forceinline__ void wide_frag(const uint8_t *slot, v4i (&af)[4], v4i (&bf)[4]) {
  const int lane = lane_id(), wave = threadIdx.x >> 6, wq = wave >> 2, wp = wave & 3;
  const int off = (lane & 15) * 64 + 16 * ((lane >> 4) ^ wide::wswz(lane & 15));
#pragma unroll
  for (int a = 0; a < 4; ++a) af[a] = *reinterpret_cast<const v4i *>(slot + (64 * wq + 16 * a) * 64 + off);
#pragma unroll
  for (int b = 0; b < 4; ++b) bf[b] = *reinterpret_cast<const v4i *>(slot + (wide::TQ + 64 * wp + 16 * b) * 64 + off);
}

__device__ __forceinline__ void wide_mma(const v4i (&af)[4], const v4i (&bf)[4], v4i (&acc)[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b], acc[a][b], 0, 0, 0);
}

// Wait until this wave's loads of the stage before the last `ahead` issued
// stages (ahead <= 3) have landed, then barrier: every wave's loads of it have
// landed and every wave is done with the previous stage's buffer.
__device__ __forceinline__ void wide_sync(int ahead) {
  asm volatile("" ::: "memory");
  if (ahead >= 3) wide::wait_vm<3 * wide::DMA>();
  else if (ahead == 2) wide::wait_vm<2 * wide::DMA>();
  else if (ahead == 1) wide::wait_vm<wide::DMA>();
  else wide::wait_vm<0>();
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's LDS reads are done
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Sorted 64-lane list (ascending keys, PAD at the end): insert key x.
__device__ __forceinline__ uint64_t list_insert(uint64_t L, uint64_t x) {
  const int lane = lane_id();
  const int pos = __popcll(__ballot(L < x));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)L, 0x138, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(L >> 32), 0x138, 0xF, 0xF, false);
  const uint64_t up = ((uint64_t)hi << 32) | lo;  // lane l: L of lane l - 1 (wave_shr:1)
  return lane < pos ? L : (lane == pos ? x : up);
}

// The list with the candidates (one per lane, ~0 = none) absorbed: the 64
// smallest keys of both, sorted.  Up to 12 candidates are inserted one at a
// time (an insertion costs about a twelfth of a sort and merge); more are
// sorted, and merged unless the list is empty.
__device__ __forceinline__ uint64_t list_absorb(uint64_t L, uint64_t cand) {
  uint64_t mask = __ballot(cand != ~0ull);
  if (mask == 0) return L;
  if (__popcll(mask) > 12) {
    if (wave_bcast_u64(L, 0) == ~0ull) return wave_sort_u64(cand);
    return merge_sorted64(L, cand);
  }
  while (mask) {
    const int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    L = list_insert(L, wave_bcast_u64(cand, j));
  }
  return L;
}

// The scan for k <= 64 on the wide tile.  Per block: one 128-query tile and
// one range of whole point tiles; the blocks of one range run on one XCD
// (they read the same point rows).  Each query's running list (the 64
// smallest keys (distance << 32 | index) so far, sorted over the lanes) lives
// in the registers of its owner wave (queries 16 w .. 16 w + 15).  Epilogue of
// a tile, once every list holds k keys: each wave compares its 64 x 64
// distances in the fragment layout with the queries' bounds and appends the
// few below to a per (query, point quarter) buffer of SUB keys; the owners
// absorb them and publish their new k-th keys.  The first tile of a range
// (lists not yet full), and the queries whose buffer overflowed, take the
// other way: each wave tile's distances are staged in LDS in turn and the
// owners absorb them one point row at a time.
//
// A query's bound is the smaller of its list's k-th key and gtau[q], the
// smallest k-th key any range has published (atomicMin).  A key above some
// range's k-th key has k smaller keys in that range, so it is not among the
// query's k nearest and may be dropped; the true k nearest all pass (a key
// equal to a published k-th key is that range's own point).  gtau is read
// back once per tile, by the same LDS loads as the stages, so a range's list
// may hold fewer than k keys at the end; the merge takes the k smallest of
// all lists.
template <int NST>
__global__ __launch_bounds__(512) void k_naive_u8_wide(const int8_t *__restrict__ Q8, const int32_t *__restrict__ qn,
                                                       const int8_t *__restrict__ X8, const int32_t *__restrict__ xn,
                                                       int64_t nq, int64_t n, int64_t mp, int k, int64_t nranges,
                                                       uint64_t *__restrict__ part, uint64_t *__restrict__ gtau) {
  using namespace wide;
  constexpr uint64_t PAD = ~0ull;
  static_assert(NST >= 3 && NST <= 4, "stages in flight: 1..2");
  __shared__ __align__(1024) uint8_t ring[NST * STAGE];
  // the candidate buffers, or (staged way, after they are read) one wave
  // tile's distances
  constexpr int CBW = TQ * 4 * SUB * 2 > 64 * WSTR ? TQ * 4 * SUB * 2 : 64 * WSTR;
  __shared__ __align__(16) uint32_t cbw[CBW];
  uint64_t(*Cb)[4 * SUB] = reinterpret_cast<uint64_t(*)[4 * SUB]>(cbw);
  uint32_t *Ds = cbw;
  __shared__ uint64_t tauq[TQ];
  __shared__ uint32_t qnl[TQ];   // |q'|^2 of the tile's queries
  // |x'|^2 of the points of the tiles in flight (tile t_lo + i in buffer i % NST:
  // at most NST tiles have a stage loaded and not yet multiplied)
  __shared__ __align__(16) uint32_t xnl[NST][TP];
  __shared__ __align__(16) uint64_t gtl[NST][TQ];  // gtau of the tile's queries, likewise per tile in flight
  __shared__ uint32_t cntq[TQ];  // byte wp: candidates of point quarter wp this tile (SUB + 1: overflow)
  __shared__ int flags[2];       // per tile parity: bit 0 some list not yet full, bit 1 overflow
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, wq = wave >> 2, wp = wave & 3, g = lane >> 4;
  const int64_t nqt = (nq + TQ - 1) / TQ;
  const int64_t j = blockIdx.x / kXcds;
  const int64_t r = (j / nqt) * kXcds + blockIdx.x % kXcds;  // point range (all its query tiles on one XCD)
  if (r >= nranges) return;
  const int64_t q0 = (j % nqt) * TQ;
  const int64_t ntile = (n + TP - 1) / TP;
  const int64_t t_lo = r * ntile / nranges, t_hi = (r + 1) * ntile / nranges;
  const int nsl = (int)(mp / BK);
  const int nst = (int)((t_hi - t_lo) * nsl);  // the block's stages
  // loads: per wave and stage one 1 KB piece of the query rows (piece
  // `wave`) and two of the point rows (pieces wave + 8, wave + 16); rows past
  // nq (n) repeat the last row, which the epilogue ignores
  const int piece = wide_piece(lane), rl = 16 * wave + (lane >> 2);
  const int8_t *asrc = Q8 + std::min<int64_t>(q0 + rl, nq - 1) * mp + piece;
  const int8_t *bsrc0 = nullptr, *bsrc1 = nullptr;
  int it = 0, isl = 0, iss = 0;  // next stage to load: tile t_lo + it, stage isl; stages loaded so far
  auto point_rows = [&]() {
    const int64_t tp = (t_lo + it) * TP;
    bsrc0 = X8 + std::min<int64_t>(tp + rl, n - 1) * mp + piece;
    bsrc1 = X8 + std::min<int64_t>(tp + 128 + rl, n - 1) * mp + piece;
  };
  const uint32_t ring_lds = lds_addr(ring), xnl_lds = lds_addr(&xnl[0][0]), gtl_lds = lds_addr(&gtl[0][0]);
  int islot = 0, ixn = 0;  // ring buffer of the next load; norm buffer of the next tile
  auto issue = [&]() {
    const uint32_t slot = ring_lds + islot * STAGE + 1024 * wave;
    const int64_t k0 = (int64_t)isl * BK;
    lds_load16(asrc + k0, slot);
    lds_load16(bsrc0 + k0, slot + 8 * 1024);
    lds_load16(bsrc1 + k0, slot + 16 * 1024);
    // with a tile's first stage, wave 0 also loads the tile's point norms
    // (the norm array is padded to whole tiles)
    if (isl == 0) {
      if (wave == 0) lds_load16(xn + (t_lo + it) * TP + 4 * lane, xnl_lds + ixn * TP * 4);
      if (wave == 1) lds_load16(gtau + q0 + 2 * lane, gtl_lds + ixn * TQ * 8);  // (gtau padded to whole tiles)
      ixn = ixn + 1 == NST ? 0 : ixn + 1;
    }
    islot = islot + 1 == NST ? 0 : islot + 1;
    ++iss;
    if (++isl == nsl) {
      isl = 0;
      ++it;
      if (t_lo + it < t_hi) point_rows();
    }
  };
  if (tid < TQ) {  // (before the first ring loads: the compiler waits for this load with vmcnt(0))
    tauq[tid] = q0 + tid < nq ? PAD : 0ull;  // nothing passes for a query past nq
    qnl[tid] = q0 + tid < nq ? (uint32_t)qn[q0 + tid] : 0u;
    cntq[tid] = 0;
  }
  point_rows();
#pragma unroll
  for (int s = 0; s < NST - 1; ++s)
    if (s < nst) issue();
  // the fragments of a stage are read one stage ahead of its products
  v4i fa[4], fb[4];
  wide_sync(iss - 1);
  wide_frag(ring, fa, fb);
  int rslot = 1;  // ring buffer of the stage after the current one
  uint64_t L[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) L[t] = PAD;
  if (tid == 0) {
    flags[0] = 1;
    flags[1] = 0;
  }
  int s = 0;
  for (int64_t t = t_lo; t < t_hi; ++t) {
    const int64_t tp0 = t * TP, pend = std::min(n, tp0 + TP);
    v4i acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};
    // stage s + 1 landed (and every wave is past stage s - 1, whose buffer
    // takes the next load); its fragments load during this stage's products.
    // After the block's last stage the read is of a stale buffer and unused.
    // Two stages per iteration, the fragment registers in alternation.
    v4i na[4], nb[4];
    auto step = [&](v4i(&ca)[4], v4i(&cb)[4], v4i(&xa)[4], v4i(&xb)[4]) {
      wide_sync(std::max(0, iss - 2 - s));
      if (iss < nst) issue();
      wide_frag(ring + rslot * STAGE, xa, xb);
      rslot = rslot + 1 == NST ? 0 : rslot + 1;
      wide_mma(ca, cb, acc);
      ++s;
    };
    int sl = 0;
    for (; sl + 1 < nsl; sl += 2) {
      step(fa, fb, na, nb);
      step(na, nb, fa, fb);
    }
    if (sl < nsl) {
      step(fa, fb, na, nb);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        fa[e] = na[e];
        fb[e] = nb[e];
      }
    }
    uint32_t xv[4];  // |x'|^2 of the lane's points (fragment columns; loaded with the tile's first stage)
    bool pok[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int pl = 64 * wp + 16 * b + (lane & 15);
      pok[b] = tp0 + pl < pend;
      xv[b] = xnl[(t - t_lo) % NST][pl];  // (buffer (t - t_lo) % NST: loaded with the tile's first stage)
    }
    uint32_t qv[4][4];  // |q'|^2 of the lane's queries (fragment rows)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) qv[a][v] = qnl[64 * wq + 16 * a + 4 * g + v];
    const uint64_t *gt = gtl[(t - t_lo) % NST];
    const int par = (int)((t - t_lo) & 1);
    const int fl0 = flags[par];  // written before the stage barriers of this tile
    uint32_t need = 0;           // owner: queries 16 wave + i that take the staged way this tile
    if (!(fl0 & 1)) {
      // screen in the fragment layout against the queries' bounds: a 32-bit
      // test of the distance first (d <= the bound's distance, a superset),
      // the exact key test only for a fragment row with a hit
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ql = 64 * wq + 16 * a + 4 * g + v;
          const uint64_t tau = std::min(tauq[ql], gt[ql]);
          const uint32_t th = (uint32_t)(tau >> 32);
          uint32_t d[4];
          bool hit = false;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            d[b] = qv[a][v] + xv[b] - 2u * (uint32_t)acc[a][b][v];
            hit = hit || (pok[b] && d[b] <= th);
          }
          if (__ballot(hit) == 0) continue;  // wave-uniform
          int cnt = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const uint64_t key = ((uint64_t)d[b] << 32) | (uint64_t)(tp0 + 64 * wp + 16 * b + (lane & 15));
            const bool pass = pok[b] && key < tau;
            const uint64_t m = __ballot(pass);
            const uint32_t gm = (uint32_t)(m >> (16 * g)) & 0xFFFFu;
            const int pre = __popc(gm & ((1u << (lane & 15)) - 1u));
            if (pass && cnt + pre < SUB) Cb[ql][SUB * wp + cnt + pre] = key;
            cnt += __popc(gm);
          }
          if ((lane & 15) == 0 && cnt > 0)
            reinterpret_cast<uint8_t *>(cntq)[4 * ql + wp] = (uint8_t)std::min(cnt, SUB + 1);
        }
      if (tid == 0) flags[par ^ 1] = 0;  // (read again two tiles on, after many barriers)
      __syncthreads();
      // owners absorb their buffers; an overflowed query takes the staged way.
      // Lane i < 16 reads the counts of query 16 wave + i.
      const uint32_t c4l = lane < 16 ? cntq[16 * wave + lane] : 0u;
      const uint64_t has = __ballot(c4l != 0);
      const uint64_t ovf = __ballot(((c4l + 0x77777777u) & 0x80808080u) != 0);  // some byte above SUB
      if (c4l != 0) cntq[16 * wave + lane] = 0;
      const int any = ovf != 0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (!((has >> i) & 1u)) continue;  // wave-uniform
        if ((ovf >> i) & 1u) {
          need |= 1u << i;
          continue;
        }
        const int ql = 16 * wave + i;
        const uint32_t c4 = (uint32_t)__builtin_amdgcn_readlane((int)c4l, i);
        // lane j < 4 SUB: entry j % SUB of quarter j / SUB
        const int sub = (lane / SUB) & 3, e = lane % SUB;
        const uint64_t cand = (lane < 4 * SUB && e < (int)((c4 >> (8 * sub)) & 255u)) ? Cb[ql][lane] : PAD;
        L[i] = list_absorb(L[i], cand);
        const uint64_t tau = wave_bcast_u64(L[i], k - 1);
        if (lane == 0) {
          tauq[ql] = tau;
          if (tau < gt[ql]) atomicMin((unsigned long long *)&gtau[q0 + ql], (unsigned long long)tau);
        }
      }
      if (any && lane == 0) atomicOr(&flags[par], 2);
      __syncthreads();
    } else {
      if (tid == 0) flags[par ^ 1] = 0;
      need = 0xFFFFu;
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (q0 + 16 * wave + i >= nq) need &= ~(1u << i);
    }
    if ((fl0 & 1) || (flags[par] & 2)) {  // block-uniform
      // the staged way: each wave tile's distances through LDS in turn
      for (int w8 = 0; w8 < 8; ++w8) {
        if (wave == w8) {
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int ql = 16 * a + 4 * g + v;
                const uint32_t d = qv[a][v] + xv[b] - 2u * (uint32_t)acc[a][b][v];
                Ds[ql * WSTR + 16 * b + (lane & 15)] = pok[b] ? d : 0xFFFFFFFFu;
              }
        }
        __syncthreads();
        if ((wave >> 2) == (w8 >> 2) && need != 0) {
          const int64_t pb = tp0 + 64 * (w8 & 3) + lane;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            if (!((need >> i) & 1u)) continue;
            const int ql = 16 * (wave & 3) + i;  // row of the staged tile
            const uint32_t d = Ds[ql * WSTR + lane];
            const uint64_t key = d == 0xFFFFFFFFu ? PAD : (((uint64_t)d << 32) | (uint64_t)pb);
            const uint64_t tau = std::min(wave_bcast_u64(L[i], k - 1), gt[16 * wave + i]);
            L[i] = list_absorb(L[i], key < tau ? key : PAD);
          }
        }
        __syncthreads();
      }
      bool full = true;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int ql = 16 * wave + i;
        const uint64_t tau = wave_bcast_u64(L[i], k - 1);
        if ((need >> i) & 1u) {
          if (lane == 0) {
            tauq[ql] = tau;
            if (tau < gt[ql]) atomicMin((unsigned long long *)&gtau[q0 + ql], (unsigned long long)tau);
          }
          full = full && std::min(tau, gt[ql]) != PAD;
        }
      }
      // a query past nq never counts against `full`
      if (!full && lane == 0) atomicOr(&flags[par ^ 1], 1);
    }
    // (the next tile's stage barriers order these LDS writes before its reads)
  }
  // the block's list per query -> part[q][range][k]
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t q = q0 + 16 * wave + i;
    if (q < nq && lane < k) part[(q * nranges + r) * (int64_t)k + lane] = L[i];
  }
}

// Merge per query: the k smallest keys over all ranges, sorted; index and
// distance out.
__global__ __launch_bounds__(1024) void k_naive_merge(const uint64_t *__restrict__ part, int64_t nranges, int k,
                                                      int64_t *__restrict__ out_idx, double *__restrict__ out_dist) {
  const int64_t q = blockIdx.x;
  const uint64_t *p = part + q * nranges * k;
  const int64_t N = nranges * k;
  __shared__ SelScratch ss;
  __shared__ uint64_t key[kMaxKH];
  __shared__ int32_t id[kMaxKH];
  __shared__ int cnt;
  int less;
  const uint64_t v = block_kth_gen<1024>(N, [&](int64_t t) { return p[t]; }, k, ss, &less);
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int64_t t = threadIdx.x; t < N; t += 1024) {
    const uint64_t kk = p[t];
    if (kk <= v) {  // keys are unique
      const int pos = atomicAdd(&cnt, 1);
      if (pos < kMaxKH) {
        key[pos] = kk;
        id[pos] = (int32_t)(kk & 0xFFFFFFFFu);
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
    out_idx[q * k + t] = (int64_t)(key[t] & 0xFFFFFFFFu);
    if (out_dist) out_dist[q * k + t] = (double)(key[t] >> 32);
  }
}

template <int KC, int MET>
static void launch_naive_u8(const int8_t *Q8, const int32_t *qn, const int8_t *X8, const int32_t *xn,
                            const knn_db_s *db, int64_t nq, int k, int64_t prange, uint64_t *part, int64_t nranges,
                            hipStream_t st) {
  dim3 grid((unsigned)nranges, (unsigned)((nq + NBQ - 1) / NBQ));
  if (k <= 64)
    hipLaunchKernelGGL(k_naive_u8_k64<MET>, grid, dim3(256), 0, st, Q8, qn, X8, xn, nq, db->n, db->mp, k, prange, part,
                       nranges);
  else
    hipLaunchKernelGGL((k_naive_u8<KC, MET>), grid, dim3(256), 0, st, Q8, qn, X8, xn, nq, db->n, db->mp, k, prange,
                       part, nranges);
}

// Working memory of one u8 scan: the shifted (or zero-padded) query rows,
// their squared norms and the per-range candidate lists.
struct NaiveU8Ws {
  int64_t prange = 0, nranges = 0;
  size_t bytes_q = 0, bytes_qn = 0, bytes_part = 0;
  size_t total() const { return bytes_q + bytes_qn + bytes_part; }
};

static NaiveU8Ws naive_u8_ws(const knn_db_s *db, int64_t nq, int32_t k, int64_t prange) {
  NaiveU8Ws w;
  w.prange = prange;
  w.nranges = (db->n + prange - 1) / prange;
  w.bytes_q = (size_t)nq * db->mp + 256;
  w.bytes_qn = sizeof(int32_t) * nq + 256;
  w.bytes_part = sizeof(uint64_t) * nq * w.nranges * k;
  return w;
}

// ws: the caller's working memory of ws_cap bytes, or nullptr (allocated
// here, stream-ordered).  With fixed memory the point ranges grow until the
// candidate lists fit (the k smallest keys do not depend on the ranges).
static int naive_u8(knn_db_s *db, const uint8_t *dq, int64_t nq, int32_t k, int64_t *out_idx, double *out_dist,
                    hipStream_t st, void *ws_fixed = nullptr, size_t ws_cap = 0) {
  const bool l1 = db->metric == KNN_METRIC_L1;
  // squared l2 distances below 2^32 (and exact int32 MFMA sums); l1 sums below 2^32
  if (!l1 && db->m > 65536) return fail(KNN_EINVAL, "naive u8 scan supports m <= 65536");
  if (l1 && db->m > 16777216) return fail(KNN_EINVAL, "naive u8 l1 scan supports m <= 2^24");
  if (k > 128) return fail(KNN_EINVAL, "naive u8 scan supports k <= 128");
  const int64_t n = db->n;
  const char *nb_env = std::getenv("KNN_NAIVE_BLOCKS");
  const char *wide_env = std::getenv("KNN_NAIVE_WIDE");
  if (!l1 && k <= 64 && !(wide_env && wide_env[0] == '0')) {
    // the wide tile: about KNN_NAIVE_BLOCKS blocks (default 256, one per CU),
    // point ranges of whole 256-point tiles
    const int64_t nqt = (nq + wide::TQ - 1) / wide::TQ, ntile = (n + wide::TP - 1) / wide::TP;
    const int64_t nblk = std::max<int64_t>(1, nb_env ? std::atoll(nb_env) : 256);
    int64_t nranges = std::max<int64_t>(1, std::min<int64_t>(ntile, (nblk + nqt - 1) / nqt));
    NaiveU8Ws w;
    w.bytes_q = (size_t)nq * db->mp + 256;
    // the query norms, then (256-byte aligned) the published k-th keys, whole
    // 128-query tiles
    const size_t qn_bytes = (sizeof(int32_t) * nq + 255) / 256 * 256;
    w.bytes_qn = qn_bytes + sizeof(uint64_t) * (size_t)nqt * wide::TQ;
    auto part_bytes = [&](int64_t nr) { return sizeof(uint64_t) * (size_t)nq * (size_t)nr * (size_t)k; };
    w.bytes_part = part_bytes(nranges);
    void *ws = ws_fixed;
    if (ws_fixed) {
      while (w.total() > ws_cap && nranges > 1) {
        nranges = (nranges + 1) / 2;
        w.bytes_part = part_bytes(nranges);
      }
      if (w.total() > ws_cap)
        return fail(KNN_EINVAL, "naive scan needs " + std::to_string(w.total()) + " bytes of working memory, more "
                                    "than the fixed " + std::to_string(ws_cap));
    } else {
      HIP_TRY(hipMallocAsync(&ws, w.total(), st));
    }
    int8_t *Q8 = (int8_t *)ws;
    int32_t *qn = (int32_t *)((uint8_t *)ws + w.bytes_q);
    uint64_t *gtau = (uint64_t *)((uint8_t *)ws + w.bytes_q + qn_bytes);
    uint64_t *part = (uint64_t *)((uint8_t *)ws + w.bytes_q + w.bytes_qn);
    int tok = prof_begin(PROF_NAIVE_REST, st);
    hipLaunchKernelGGL(k_prep_u8_queries, dim3((unsigned)nq), dim3(256), 0, st, dq, db->m, db->mp, Q8, qn);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)nqt), dim3(wide::TQ), 0, st, gtau, ~0ull);
    prof_end(tok, st, 0.0);
    tok = prof_begin(PROF_NAIVE_GEMM, st);
    const int64_t nblocks = (nranges + kXcds - 1) / kXcds * kXcds * nqt;
    // LDS ring stages (KNN_NAIVE_STAGES: 3 or 4 (default); NST - 2 in flight
    // during a stage's products)
    const char *ns_env = std::getenv("KNN_NAIVE_STAGES");
    const int nstages = ns_env ? std::atoi(ns_env) : 4;
#define KNN_WIDE_LAUNCH(NST_)                                                                                  \
  hipLaunchKernelGGL(k_naive_u8_wide<NST_>, dim3((unsigned)nblocks), dim3(512), 0, st, Q8, qn, db->xs8,       \
                     db->norm_i, nq, n, db->mp, k, nranges, part, gtau)
    if (nstages == 3) KNN_WIDE_LAUNCH(3);
    else KNN_WIDE_LAUNCH(4);
#undef KNN_WIDE_LAUNCH
    prof_end(tok, st, 2.0 * (double)nq * (double)n * (double)db->m);
    tok = prof_begin(PROF_NAIVE_REST, st);
    hipLaunchKernelGGL(k_naive_merge, dim3((unsigned)nq), dim3(1024), 0, st, part, nranges, k, out_idx, out_dist);
    prof_end(tok, st, 0.0);
    HIP_TRY(hipGetLastError());
    if (!ws_fixed) HIP_TRY(hipFreeAsync(ws, st));
    return KNN_OK;
  }
  const int64_t qt = (nq + NBQ - 1) / NBQ;
  // about KNN_NAIVE_BLOCKS blocks in all (default 512: two per CU, one
  // wave of blocks); longer point ranges amortise each block's first tiles,
  // where every distance still enters the running lists
  const int64_t nblk = std::max<int64_t>(1, nb_env ? std::atoll(nb_env) : 512);
  int64_t prange = (n * qt + nblk - 1) / nblk;
  prange = std::max<int64_t>(NBP, (prange + NBP - 1) / NBP * NBP);
  NaiveU8Ws w = naive_u8_ws(db, nq, k, prange);
  void *ws = ws_fixed;
  if (ws_fixed) {
    while (w.total() > ws_cap && w.nranges > 1) {
      prange = (prange * 2 + NBP - 1) / NBP * NBP;
      w = naive_u8_ws(db, nq, k, std::min<int64_t>(prange, (n + NBP - 1) / NBP * NBP));
    }
    if (w.total() > ws_cap)
      return fail(KNN_EINVAL, "naive scan needs " + std::to_string(w.total()) + " bytes of working memory, more than "
                                  "the fixed " + std::to_string(ws_cap));
  } else {
    HIP_TRY(hipMallocAsync(&ws, w.total(), st));
  }
  prange = w.prange;
  const int64_t nranges = w.nranges, mp = db->mp;
  int8_t *Q8 = (int8_t *)ws;
  int32_t *qn = (int32_t *)((uint8_t *)ws + w.bytes_q);
  uint64_t *part = (uint64_t *)((uint8_t *)ws + w.bytes_q + w.bytes_qn);
  int tok = prof_begin(PROF_NAIVE_REST, st);
  if (l1)  // zero-padded u8 query rows
    hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)nq), dim3(256), 0, st, dq, nq, db->m, mp, 1, (uint8_t *)Q8);
  else
    hipLaunchKernelGGL(k_prep_u8_queries, dim3((unsigned)nq), dim3(256), 0, st, dq, db->m, mp, Q8, qn);
  prof_end(tok, st, 0.0);
  tok = prof_begin(PROF_NAIVE_GEMM, st);
  if (l1)
    launch_naive_u8<128, KNN_METRIC_L1>(Q8, nullptr, (const int8_t *)db->xpad, nullptr, db, nq, k, prange, part,
                                        nranges, st);
  else
    launch_naive_u8<128, KNN_METRIC_L2>(Q8, qn, db->xs8, db->norm_i, db, nq, k, prange, part, nranges, st);
  // work units: 2 operations per (query, point, coordinate) -- a multiply-add,
  // or an absolute difference and its addition
  prof_end(tok, st, 2.0 * (double)nq * (double)n * (double)db->m);
  tok = prof_begin(PROF_NAIVE_REST, st);
  hipLaunchKernelGGL(k_naive_merge, dim3((unsigned)nq), dim3(1024), 0, st, part, nranges, k, out_idx, out_dist);
  prof_end(tok, st, 0.0);
  HIP_TRY(hipGetLastError());
  if (!ws_fixed) HIP_TRY(hipFreeAsync(ws, st));
  return KNN_OK;
}

// ------------------------------------------------- allocation-free scan

// Fixed working memory of knn_naive_noalloc: one array per device for the
// life of the process.  Host code never passes `scratch` itself to a kernel
// (in host code the name is a host-side stand-in); it passes the device
// address that hipGetSymbolAddress returns, looked up once per device.
constexpr size_t kNoallocScratch = (size_t)KNN_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) uint8_t scratch[kNoallocScratch];

static int scratch_address(void **out) {
  static std::mutex mu;
  static std::map<int, void *> addr;  // device -> address of its copy of the array
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(KNN_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    it = addr.emplace(dev, p).first;
  }
  *out = it->second;
  return KNN_OK;
}

// The exact scan for k above the fused top-k lists' capacity (k up to
// KNN_MAX_KH): one block per query.  Each point's distance in integers (a
// wave per point: coalesced row reads, four bytes a lane per step, the
// query row from the caches), its key (distance << 32 | index) in scratch,
// the k-th smallest key by radix selection, then the k keys at or below it
// (distinct: the index is part of the key) sorted -- the (distance, index)
// order of the fused scan.
template <int MET>
__global__ __launch_bounds__(1024) void k_naive_u8_full(const uint8_t *__restrict__ X, const uint8_t *__restrict__ Q,
                                                        int64_t n, int64_t m, int k, int64_t q0,
                                                        uint64_t *__restrict__ scratch, int64_t *__restrict__ out_idx,
                                                        double *__restrict__ out_dist) {
  const int64_t q = q0 + blockIdx.x;
  uint64_t *keys = scratch + (int64_t)blockIdx.x * n;
  const uint8_t *qv = Q + q * m;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const bool words = (m & 3) == 0;
  for (int64_t i = wave; i < n; i += 1024 / kWave) {
    const uint8_t *row = X + i * m;
    uint32_t acc = 0;  // below 2^32: m <= 65536 (squared l2) or m <= 2^24 (l1)
    if (words) {
      const uint32_t *r4 = reinterpret_cast<const uint32_t *>(row), *q4 = reinterpret_cast<const uint32_t *>(qv);
      for (int64_t w = lane; w < m / 4; w += kWave) {
        const uint32_t xv = r4[w], qw = q4[w];
        if constexpr (MET == KNN_METRIC_L1) {
          acc += __builtin_amdgcn_sad_u8(xv, qw, 0u);
        } else {
          acc += __builtin_amdgcn_udot4(xv, xv, 0u, false) + __builtin_amdgcn_udot4(qw, qw, 0u, false) -
                 2u * __builtin_amdgcn_udot4(xv, qw, 0u, false);
        }
      }
    } else {
      for (int64_t j = lane; j < m; j += kWave) {
        const int d = (int)row[j] - (int)qv[j];
        acc += MET == KNN_METRIC_L1 ? (uint32_t)(d < 0 ? -d : d) : (uint32_t)(d * d);
      }
    }
    for (int o = kWave / 2; o > 0; o >>= 1) acc += (uint32_t)__shfl_xor((int)acc, o);
    if (lane == 0) keys[i] = ((uint64_t)acc << 32) | (uint64_t)i;
  }
  __syncthreads();
  __shared__ SelScratch ss;
  __shared__ uint64_t key[kMaxKH];
  __shared__ int32_t id[kMaxKH];
  __shared__ int cnt;
  int less;
  const uint64_t v = block_kth_gen<1024>(n, [&](int64_t i) { return keys[i]; }, k, ss, &less);
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const uint64_t kk = keys[i];
    if (kk <= v) {
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
    out_idx[q * k + t] = (int64_t)(key[t] & 0xFFFFFFFFu);
    if (out_dist) out_dist[q * k + t] = (double)(key[t] >> 32);
  }
}

static int naive_u8_full(knn_db_s *db, const uint8_t *dq, int64_t nq, int32_t k, int64_t *out_idx,
                         double *out_dist, hipStream_t st) {
  const bool l1 = db->metric == KNN_METRIC_L1;
  if (!l1 && db->m > 65536) return fail(KNN_EINVAL, "naive u8 scan supports m <= 65536");
  if (l1 && db->m > 16777216) return fail(KNN_EINVAL, "naive u8 l1 scan supports m <= 2^24");
  const int64_t n = db->n, m = db->m;
  // queries per launch: their keys fit in 1 GiB of scratch
  const int64_t batch = std::max<int64_t>(1, std::min<int64_t>(nq, (1ll << 30) / (n * 8)));
  uint64_t *scratch = nullptr;
  HIP_TRY(hipMallocAsync(&scratch, sizeof(uint64_t) * n * batch, st));
  const int tok = prof_begin(PROF_NAIVE_GEMM, st);
  for (int64_t q0 = 0; q0 < nq; q0 += batch) {
    const unsigned cnt = (unsigned)std::min<int64_t>(batch, nq - q0);
    if (l1)
      hipLaunchKernelGGL(k_naive_u8_full<KNN_METRIC_L1>, dim3(cnt), dim3(1024), 0, st, db->X, dq, n, m, (int)k, q0,
                         scratch, out_idx, out_dist);
    else
      hipLaunchKernelGGL(k_naive_u8_full<KNN_METRIC_L2>, dim3(cnt), dim3(1024), 0, st, db->X, dq, n, m, (int)k, q0,
                         scratch, out_idx, out_dist);
  }
  prof_end(tok, st, (l1 ? 2.0 : 3.0) * (double)nq * (double)n * (double)m);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipFreeAsync(scratch, st));
  return KNN_OK;
}

int naive_run_noalloc(knn_db_s *db, const void *dq, int64_t nq, int32_t k, int64_t *out_idx, double *out_dist,
                      hipStream_t st) {
  if (db->dtype != KNN_U8) return fail(KNN_EINVAL, "knn_naive_noalloc supports u8 DBs only");
  void *ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc != KNN_OK) return rc;
  return naive_u8(db, (const uint8_t *)dq, nq, k, out_idx, out_dist, st, ws, kNoallocScratch);
}

int naive_run(knn_db_s *db, const void *dq, int64_t nq, int32_t k, int64_t *out_idx, double *out_dist,
              hipStream_t st) {
  if (db->dtype == KNN_U8)
    return k > 128 ? naive_u8_full(db, (const uint8_t *)dq, nq, k, out_idx, out_dist, st)
                   : naive_u8(db, (const uint8_t *)dq, nq, k, out_idx, out_dist, st);
  return naive_f32(db, (const float *)dq, nq, k, out_idx, out_dist, st);
}

}  // namespace knn
