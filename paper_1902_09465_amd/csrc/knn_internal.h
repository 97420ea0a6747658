// knn_internal.h -- structures shared by the host runtime and the kernels of
// libknn.  Device-resident structs are plain data (no pointers to host memory).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/knn.h"

namespace knn {

constexpr int kMaxRounds = KNN_MAX_ROUNDS;
constexpr int kPmMaxK1 = 128;  // point-major batches: k + 1 <= kPmMaxK1 (selection lists of two wave registers)
constexpr int kMaxKH = KNN_MAX_KH;

// Point flags (per query, per point).  The dump format of
// knn_adaptive_state uses the same bits.
constexpr uint8_t FL_EXACT = 1;
constexpr uint8_t FL_ACC = 2;
constexpr uint8_t FL_DISC = 4;

// Round schedule and widths of one parameter set (host-computed).
struct Sched {
  int32_t R;                      // number of sampled rounds; round R is exact
  int32_t pad;
  int32_t T[kMaxRounds];          // cumulative sample target of round r
  double alpha[kMaxRounds];       // confidence width at T[r]
};

// One query as submitted (device table, filled by the host and, for the
// f32 range scaling, by k_prep_queries).
struct QDesc {
  const void *q;        // [m] query vector
  uint64_t seed;
  int32_t k, kh;        // k and k+h
  int32_t c_exact;
  int32_t sched;        // index into the Sched table
  double W;             // sample normaliser: samples s/W lie in [0,1]
  int32_t F;            // f32 fixed-point shift (0 for u8)
  int32_t trivial;      // 1: k+h >= n or zero range -> return the first min(n,k+h) indices
  int32_t norepl;       // 1: coordinates drawn without replacement
  int32_t shared;       // 1: one coordinate sequence for all points (counter words (0, 2) / (0, 3))
  int32_t pad0;
  int64_t *out_idx;     // row of out_stride int64
  int32_t *out_count;
  knn_stats *out_stats;
  int64_t out_stride;
};

// One in-flight query (a "slot").  All slots advance one round per step.
struct Slot {
  int32_t state;        // 0 idle, 1 running
  int32_t qi;           // query index in the QDesc table
  int32_t cur;          // current round index (0..R); round R is exact
  int32_t par;          // which half of the double-buffered lists is current
  int32_t implicit;     // 0: the sets are the lists act/xa/acc; 1: round 0, every point
                        // undecided (identity); 2: the sets are given by the flags alone
                        // (points 0..n-1 filtered by flag; no lists kept)
  int32_t n_act, n_xa, n_acc;   // current list sizes
  int32_t nn_act, nn_xa, nn_acc; // sizes being built by k_decide
  int32_t k, kh, R, c_exact;
  int32_t F, norepl;
  int32_t shared, pad2;  // shared: one coordinate sequence for all points
  uint64_t seed;
  double W;
  const void *q;
  double U, L1, L2;     // thresholds of the current snapshot
  int64_t sthr[4];      // point-major batches: the same decisions as integer sums S of the
                        // round (S > sthr[0] discard, else S <= sthr[1] accept for a sampled
                        // pair; sthr[2], sthr[3] for an exact pair), set with U, L1, L2
  int64_t coord_evals, exact_points;
  int32_t rounds;
  int32_t pm_copy;      // point-major batches: 1 in the step where the slot turned sparse (its sums
                        // are then copied slot-major by k_pm_to_slot after k_finish)
  int32_t T[kMaxRounds];
  double alpha[kMaxRounds];
};

// A sampled round that every running slot of a launch shares (query-lane
// sampling): the common seed, the round's sample range [t0, t1) and index.
struct QlRound {
  uint64_t seed;
  uint32_t t0, t1;
  int32_t cur;
  int32_t impl;         // 1: round 0, every point undecided
  int32_t exact;        // 1: the exact round (t0, t1, seed unused)
  int32_t norepl;       // 1: coordinates drawn without replacement
  int32_t shared;       // 1: one coordinate sequence for all points
  int32_t pad;
};

// A point-major batch whose queries share one coordinate sequence
// (sampling 2 or 3, one seed): the sequence and the points and queries
// gathered at its coordinates, so that a round's samples are a range of
// columns of these copies.
struct SeqBufs {
  uint32_t *js = nullptr;  // [kp] coordinate of sample t (~0u past the samples held)
  int8_t *xs = nullptr;    // [n][kp] points at the sequence's coordinates (x - 128; l1: raw bytes)
  int8_t *qs = nullptr;    // [nqp][kp] the queries, likewise (rows of idle slots zero)
  int32_t *xn = nullptr;   // [nb][n] squared norms of the xs rows over the samples t < T'_b (l2)
  int32_t *qn = nullptr;   // [nb][nqp] the same for the qs rows
  float *xf = nullptr;     // fp32 DBs: [n][kp] points at the sequence's coordinates (no xs, qs, norms)
  float *qf = nullptr;     // fp32 DBs: [nslots][kp] the slots' queries, likewise
  int32_t *flag = nullptr;  // device word: whether the exact round's columns are needed (set per batch)
  int64_t kp = 0;          // row length, a multiple of 64
  int32_t tlen = 0;        // samples held: the last sampled target, or m without replacement
  int32_t nb = 0;          // boundaries T'_0 = 0, T'_b = T[b-1] (b <= R), and T'_{R+1} = m
                           // without replacement
};

// Engine control block (device).
struct Ctl {
  int32_t next_query;   // admission cursor (monotone)
  int32_t done;         // finished queries
  int32_t nq;           // queries submitted so far (the host may raise it between steps)
  int32_t stop_after;   // > 0: debug stop after that many decide steps (no output)
  int32_t qcap;         // QDesc/Sched tables are rings of qcap entries (query qi at qi % qcap)
  int32_t run_hi;       // packed admission: 1 + the highest slot running after the last admission
  int32_t pad[2];
};

// Device buffers of one engine instance (per-slot arrays are [nslots][n]).
struct Bufs {
  int64_t *S;           // running sums
  uint8_t *fl;          // flags
  uint8_t *ri;          // round index of last sampled target
  int32_t *act;         // [nslots][2][n] undecided, still sampled
  int32_t *xa;          // [nslots][2][n] undecided, exact
  int32_t *acc;         // [nslots][n] accepted
  uint64_t *part;       // [nslots][part_stride] per-chunk selection candidates
  int64_t part_stride;
  int32_t *cand;        // [nslots][kMaxKH] candidate-exact picks
  uint32_t *dpm;        // query-lane batches: D, point-major [n][dpm_stride] (running sums when
                        // Geometry::flagsets); nullptr otherwise
  int64_t dpm_stride;
};

struct Geometry {
  int64_t n, m;
  int32_t dtype;        // KNN_U8 / KNN_F32
  int32_t nslots;
  int32_t ch_sample;    // points per sample block
  int32_t ch_select;    // elements per selection block
  int32_t ch_decide;    // elements per decide block
  int32_t lpp;          // lanes per point in sampled rounds
  uint64_t *prof;       // NULL, or work counters: [0] algorithmic bytes, [1] samples, [2] exact
                        // elements, [3] distinct Philox draws x 4
  const int8_t *x8;     // u8 DB: x - 128 as int8, [n][mp] (exact round on the matrix cores);
                        // l1: the points' bytes zero-padded to [n][mp] (exact round by v_sad_u8 tiles)
  const int32_t *xn;    // u8 DB: sum (x - 128)^2 per row
  int64_t mp;           // m padded to a multiple of 64
  int32_t grouped;      // 1: sample GRP slots per block when they share seed and round
  int32_t stage;        // grouped sampled rounds: point rows per LDS tile (0: gather from HBM)
  int32_t kmax;         // largest k of the slots' queries
  int32_t metric;       // KNN_METRIC_L2 (samples (x_ij - x_j)^2) or KNN_METRIC_L1 (|x_ij - x_j|)
  int32_t flagsets;     // 1: point-major batch: dense slots (implicit 1/2) keep their sums
                        // point-major and their sets in the flags; sparse slots (implicit 0)
                        // use the per-slot list kernels
  int32_t nslots_all;   // slots of the engine; nslots may be lower for a step (packed admission:
                        // every running slot lies below nslots)
  int32_t packed_admit; // 1: queries are admitted into the lowest idle slots by k_admit_packed
                        // (one block, after k_finish), which also reports Ctl::run_hi
  int32_t sparse_div;   // a dense slot turns sparse once its undecided count is <= n / sparse_div
                        // (0: never)
};

// Order-preserving map of a non-NaN double to uint64 (and back).
__host__ __device__ inline uint64_t dkey(double x) {
  if (x == 0.0) x = 0.0;  // canonical +0
  uint64_t b;
  __builtin_memcpy(&b, &x, 8);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ inline double dkey_inv(uint64_t k) {
  uint64_t b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  double x;
  __builtin_memcpy(&x, &b, 8);
  return x;
}

}  // namespace knn
