// knn_host.h -- host runtime internals of libknn (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>

#include "knn_internal.h"

namespace knn {
struct Plan;
void plan_free(Plan *p);
// Performance knobs (never result-defining); see knobs_for.
struct Knobs {
  int32_t valid = 0;        // set by the autotuner
  int32_t ql = 1;           // query-lane sampling allowed
  int32_t ql_min = 64;      // ... from this many slots
  int32_t group = 1;        // 16-slot grouped sampling allowed
  int32_t lpp = 0;          // lanes per point of the grouped kernel (0: per round)
  int32_t ch_sample = 2048; // points per sampling block
  int32_t stage_min = 1 << 30;  // LDS-staged rows from this round size (off)
  int32_t stage_rows = 8;
  int32_t graph = 1;        // capture and replay repeated batches
  int32_t sparse_div = 16;  // point-major batches: slots with <= n / sparse_div undecided points switch
                            // to per-slot lists (0: never)
  int32_t seq = 1;          // shared coordinate sequences: rounds over gathered copies allowed
};
}  // namespace knn

struct knn_db_s {
  const uint8_t *X = nullptr;  // [n][m] point-major (u8 or f32 bytes)
  void *owned = nullptr;       // library allocation when copied
  int64_t n = 0, m = 0;
  int32_t dtype = KNN_U8;
  int32_t metric = KNN_METRIC_L2;
  double lo = 0.0, hi = 0.0;   // f32 value range over all points
  // naive-scan auxiliaries
  int8_t *xs8 = nullptr;       // u8: x - 128 as int8, [n][mp] (mp = m padded to 64)
  int64_t mp = 0;
  int32_t *norm_i = nullptr;   // u8: sum (x-128)^2 per row
  uint16_t *xbf = nullptr;     // f32: split BF16 copy, hi [n][mp] then lo [n][mp]
  float *norm_f = nullptr;     // f32: |x|^2 per row (fp64 sum rounded to fp32)
  float *rownorm = nullptr;    // f32: |x| per row (for the error bound)
  void *xpad = nullptr;        // l1: the points with rows zero-padded to mp (u8 or f32)
  std::atomic<int> users{0};   // sessions holding the DB
  std::mutex mu;
  knn::Plan *plan = nullptr;   // cached engine + captured graph of the last batch shape
  knn::Knobs tune;             // autotuned knobs (tune.valid)
  // pinned staging of an eager batch's control block, query descriptors and
  // schedules: reused once the previous batch's copies out of it are done
  void *stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t stage_done = nullptr;
  std::mutex stage_mu;
};

namespace knn {

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// Host computation of the round schedule and widths (Section 4 footnote,
// Lemma 3, Section 5); returns false on invalid parameters.
bool host_schedule(const knn_params &p, int64_t n, int64_t m, Sched &out, std::string &why);

// A slot engine: device state for `ns` in-flight queries on one DB, plus
// QDesc/Sched rings of qcap entries.  Used by knn_adaptive (ring = the whole
// query table) and by the serving session (ring refilled while running).
struct Engine {
  knn_db_s *db = nullptr;
  hipStream_t st = nullptr;
  void *base = nullptr;
  bool async_alloc = false;
  Slot *slots = nullptr;
  Ctl *ctl = nullptr;
  QDesc *qd = nullptr;
  Sched *sched = nullptr;
  Bufs B{};
  Geometry G{};
  int64_t ns = 0, qcap = 0, nsched = 0;
  uint8_t *qt = nullptr;  // query-lane sampling: transposed queries [m][nqp] (nullptr: not used)
  uint32_t *qsum = nullptr;  // query-lane sampling: round totals [n][nqp] u32, then flags [n][nqp] u8
  int8_t *q8 = nullptr;      // query-lane exact round: shifted int8 queries [nqp][mp] (u8 DBs; l1: the
                             // queries' bytes, zero-padded)
  int32_t *q8n = nullptr;    // ... and their squared norms [nqp] (squared l2)
  int32_t nqp = 0;
  SeqBufs seq;               // one coordinate sequence for all points: its gathered copies (seq.xs null: none)
};
size_t engine_slot_bytes(int64_t n, int32_t kmax, int32_t cmax);
// seq_tlen > 0: also the gathered copies of a shared coordinate sequence
// holding seq_tlen samples, with seq_nb norm boundaries
int engine_create(Engine &E, knn_db_s *db, int64_t ns, int32_t kmax, int32_t cmax, int64_t qcap, int64_t nsched,
                  hipStream_t st, bool async_alloc, bool grouped, bool query_lane = false, int32_t seq_tlen = 0,
                  int32_t seq_nb = 0);
int engine_destroy(Engine &E);
void engine_step(Engine &E, bool any_cexact, int sample_kind = 0, int stage_rows = 0, const QlRound *ql = nullptr);
// rows per LDS tile for grouped sampled rounds of an m-dimensional DB (0: none fits)
int stage_rows_for(int64_t m, int64_t mp, int want);
Knobs knobs_for(const knn_db_s *db);
// Host-side parameter check + per-query descriptor (no device pointers for the
// query/outputs are filled here).
int make_qdesc(const knn_db_s *db, int32_t k, const knn_params &p, QDesc &d, Sched &sc);

// kernels (k_adaptive.hip)
void launch_prep_f32(QDesc *qd, int32_t nq, int64_t n, int64_t m, double lo, double hi, int32_t metric,
                     hipStream_t st);
void launch_step(Slot *slots, const QDesc *qd, const Sched *sched, Ctl *ctl, const uint8_t *X,
                 const Bufs &B, const Geometry &G, bool any_cexact, hipStream_t st, int sample_kind = 0,
                 int stage_rows = 0, const QlRound *ql = nullptr, const uint8_t *qt = nullptr, int32_t nqp = 0,
                 uint32_t *qd_buf = nullptr, const int8_t *q8 = nullptr, const int32_t *q8n = nullptr,
                 const SeqBufs *seq = nullptr);
// The shared sequence's coordinates, the queries' rows at them with their
// prefix norms at every round boundary, and the points' rows at columns
// [0, ca) (a multiple of 64, or kp) with their norms at boundaries b < ba.
void launch_seq_prepare(const Slot *slots, const Sched *sc, int32_t ns, int32_t nqp, const uint8_t *X, int64_t n,
                        int64_t m, uint64_t seed, int32_t norepl, int32_t metric, const SeqBufs &q,
                        const int32_t *xnorm, const int32_t *qnorm, int64_t ca, int32_t ba, hipStream_t st);
// The points' rows at columns [c0, c1) and their norms at boundaries
// b0 <= b < b1, when (checked on the device) some slot is running, or with
// `dense` some running slot is dense.
void launch_seq_gather_more(const Slot *slots, int32_t ns, const Sched *sc, const uint8_t *X, int64_t n, int64_t m,
                            int32_t metric, const SeqBufs &q, int64_t c0, int64_t c1, int32_t b0, int32_t b1,
                            int32_t dense, const int32_t *xnorm, hipStream_t st);
void launch_seq_prepare_f32(const Slot *slots, int32_t ns, const float *X, int64_t n, int64_t m, uint64_t seed,
                            int32_t norepl, const SeqBufs &q, hipStream_t st);
void launch_round_seq_u8(const Slot *slots, const SeqBufs &q, int32_t lo, int32_t hi, int64_t t0, int64_t t1,
                         const uint8_t *A, uint32_t *D, int32_t nqp, const Bufs &B, const Geometry &G, int32_t cur,
                         int32_t impl, int32_t exact, hipStream_t st);
void launch_build_qt(const Slot *slots, int32_t ns, int64_t m, int32_t nqp, uint8_t *qt, hipStream_t st);
void launch_build_q8(const Slot *slots, int32_t ns, int64_t m, int64_t mp, int8_t *Q8, int32_t *qn, int32_t metric,
                     hipStream_t st);
void launch_exact_ql_u8(const Slot *slots, const int8_t *Q8, const int32_t *qn, const int8_t *X8, const int32_t *xn,
                        const Bufs &B, const Geometry &G, int32_t cur, int32_t impl, uint32_t *Dpm, int32_t nqp,
                        hipStream_t st);
void launch_admit(Slot *slots, const QDesc *qd, const Sched *sched, Ctl *ctl, const uint8_t *X,
                  const Bufs &B, const Geometry &G, hipStream_t st, bool direct = false);
int64_t part_words(int64_t n, int32_t kmax, int32_t cmax);

// kernels (k_naive.hip)
int naive_prepare_db(knn_db_s *db, hipStream_t st);
int naive_run(knn_db_s *db, const void *dq, int64_t nq, int32_t k, int64_t *out_idx, double *out_dist,
              hipStream_t st);
void naive_free_db(knn_db_s *db);
// knn_naive_noalloc: u8 scan in the fixed per-device working memory
int naive_run_noalloc(knn_db_s *db, const void *dq, int64_t nq, int32_t k, int64_t *out_idx, double *out_dist,
                      hipStream_t st);
// rows of elem-byte values copied with zero padding from m to mp elements (the l1 scans' operands)
void launch_pad_rows(const uint8_t *X, int64_t rows, int64_t m, int64_t mp, int elem, uint8_t *out, hipStream_t st);
// k_naive_f32.hip
int naive_prepare_db_f32(knn_db_s *db, hipStream_t st);
int naive_f32(knn_db_s *db, const float *dq, int64_t nq, int32_t k, int64_t *out_idx, double *out_dist,
              hipStream_t st);
int db_range_f32(const float *X, int64_t count, double *lo, double *hi, hipStream_t st);

}  // namespace knn

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return knn::fail(_e == hipErrorOutOfMemory ? KNN_ENOMEM : KNN_EDEVICE,           \
                       std::string(#expr) + ": " + hipGetErrorString(_e));             \
  } while (0)
