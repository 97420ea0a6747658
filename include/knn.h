/*
 * knn.h -- C ABI of libknn: adaptive k-nearest-neighbour search on MI355X
 * (gfx950), after LeJeune, Baraniuk, Heckel, "Adaptive Estimation for
 * Approximate k-Nearest-Neighbor Computations" (AISTATS 2019).
 *
 * Conventions for every entry point:
 *  - Plain pointers and sizes only.  "dev_" pointers are device (HBM)
 *    addresses, "host_" pointers are host addresses.  The caller owns every
 *    buffer it passes and keeps it alive until the call's work is finished
 *    (stream-ordered calls: until the stream is synchronised).
 *  - Matrices are row-major: points are rows ("point-major"), X[i*m + j].
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Return value: KNN_OK (0), KNN_PENDING (1) or a negative KNN_E* code.
 *    Arguments are checked before any work is enqueued; on error nothing is
 *    enqueued and knn_last_error() describes the failure (thread-local).
 *    No C++ exception crosses the ABI.
 *  - Working memory of a batch comes from a stream-ordered pool per device
 *    that the library keeps for the life of the process (memory freed by a
 *    batch is reused by the next instead of being unmapped), plus one
 *    pinned host staging buffer per DB, freed by knn_db_destroy.
 */
#ifndef KNN_H
#define KNN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KNN_OK 0
#define KNN_PENDING 1
#define KNN_EINVAL (-1)   /* invalid argument */
#define KNN_ENOMEM (-2)   /* device or host allocation failed */
#define KNN_EDEVICE (-3)  /* HIP runtime error */
#define KNN_EBUSY (-4)    /* object still in use */
#define KNN_ENOTFOUND (-5)/* unknown ticket / id */

typedef enum { KNN_U8 = 0, KNN_F32 = 1 } knn_dtype;

#define KNN_DB_BORROW 0   /* alias dev_points; caller keeps it alive until destroy */
#define KNN_DB_COPY 1     /* copy dev_points into library-owned HBM */
#define KNN_DB_L1 2       /* flag bit: the DB's distance is l1, sum_j |x_j - y_j| (Section 3
                             notes that the results carry over to it); without it the
                             distance is the squared l2 of Section 3 */

/* Distance of a DB (knn_db_metric). */
typedef enum { KNN_METRIC_L2 = 0, KNN_METRIC_L1 = 1 } knn_metric;

#define KNN_MAX_KH 2048   /* largest k + h (adaptive) and k (naive) */
#define KNN_MAX_ROUNDS 48 /* longest round schedule */

typedef struct knn_db_s *knn_db;
typedef struct knn_session_s *knn_session;

/* Result-defining parameters of one adaptive query.  Fields marked "0 ->"
 * take the stated default when zero. */
typedef struct {
  int64_t h;           /* slack: returned set has at most k+h points; < 0 means h = k
                          (Section 4.2 takes h = k) */
  double delta;        /* failure probability in (0,1) (Theorem 1) */
  uint64_t seed;       /* Philox key; the same seed gives the same result alone or batched */
  int32_t alpha_kind;  /* 0: Section 4 footnote width (falls back to 1 when delta/n >= 0.05);
                          1: Lemma 3 width, valid for any delta;
                          2: Section 5 width sqrt(c_alpha log(1+(1+log u) n/delta)/u), no guarantee */
  double c_alpha;      /* only for alpha_kind 2, > 0 */
  int32_t b0;          /* samples per point in round 0, multiple of 4 (0 -> 64) */
  float growth;        /* target growth g >= 1: T += max(4, ceil4(ceil(T (g-1)))) (0 -> 2) */
  float theta_exact;   /* a point goes exact once the next target reaches ceil(theta m) (0 -> 1) */
  int32_t c_exact;     /* >= 0; the c_exact undecided points with the smallest estimate are
                          made exact after every sampling step (0 = pure round form) */
  int32_t sampling;    /* coordinates of the samples (Section 4):
                          0: drawn with replacement, sample t of point i from output t mod 4
                          of Philox4x32-10(key seed, counter (t/4, 0, i, 0)), coordinate
                          floor(r m / 2^32);
                          1: without replacement (Section 4 footnote): sample t < m of point i
                          is pi(t) for a per-(seed, point) permutation pi of [0, m) -- a
                          four-round Feistel network on 2h bits (2^2h >= m, h >= 1) with
                          round keys Philox4x32-10(seed, counter (0, 0, i, 1)) and round
                          function F(k, v) = lowbias32(v xor k) mod 2^h, cycle-walked into
                          [0, m) (Black & Rogaway); d^ at T = m is then the exact distance,
                          and an exact distance costs the m - T coordinates not yet seen;
                          2, 3: as 0 and 1, but one coordinate sequence j_1, j_2, ... serves
                          every point (counter words (0, 2) for the draws, (0, 3) for the
                          round keys).  Each point's samples are still i.i.d. (2) or a
                          uniform permutation (3), which is all Lemma 3 uses, so the
                          guarantee of Theorem 1 is unchanged.  Queries that share seed and
                          schedule then share every sampled coordinate, and their sampled
                          rounds run as int8 matrix products over the gathered coordinates */
} knn_params;

/* Per-query statistics (24 bytes). */
typedef struct {
  int64_t coord_evals;  /* coordinate evaluations: samples + m per exact distance (without
                           replacement: + the m - T coordinates not yet sampled) */
  int32_t rounds;       /* decide steps executed */
  int32_t count;        /* size of the returned set */
  int64_t exact_points; /* points whose distance was computed exactly */
} knn_stats;

/* Fills *p with the defaults: h = -1 (h = k), delta = 0.01, seed = 0,
 * alpha_kind = 0, c_alpha = 0, b0 = 64, growth = 2, theta_exact = 1, c_exact = 0,
 * sampling = 0. */
void knn_params_default(knn_params *p);

/* Thread-local description of the last error on this thread ("" if none). */
const char *knn_last_error(void);

/* Library version string. */
const char *knn_version(void);

/* ---------------------------------------------------------------- DB --- */

/* Registers n points of dimension m (Section 3: the point set X in R^m).
 * dev_points: device, [n][m] row-major, u8 or f32.  flags: KNN_DB_BORROW
 * aliases it, KNN_DB_COPY copies it; or-ing in KNN_DB_L1 makes every search
 * on the DB use the l1 distance (adaptive samples |x_ij - x_j|, normalised
 * by 255 for u8 and by the value range for f32; the naive scan sums
 * |x_j - q_j|).  Precomputes for the naive scan: squared l2 -- row norms,
 * shifted int8 (u8) or split BF16 (f32) copies; l1 -- a copy with rows
 * zero-padded to a multiple of 64 elements.  For f32 also the value range.
 * Synchronous.  Errors: EINVAL (n < 1, m < 1, n >= 2^31, bad dtype/flags,
 * NULL), ENOMEM, EDEVICE. */
int knn_db_create(const void *dev_points, int64_t n, int64_t m, knn_dtype dt,
                  int32_t flags, knn_db *out);

/* Releases the DB.  EBUSY while a session still holds it or requests on it
 * are pending.  Waits for the library's own work on it to finish. */
int knn_db_destroy(knn_db db);

/* n, m and dtype of a DB. */
int knn_db_info(knn_db db, int64_t *n, int64_t *m, int32_t *dtype);

/* The DB's distance: KNN_METRIC_L2 (squared l2) or KNN_METRIC_L1. */
int knn_db_metric(knn_db db, int32_t *metric);

/* ---------------------------------------------------------- adaptive --- */

/* Round schedule and widths that knn_adaptive uses for one parameter set on
 * a DB with n points of dimension m (Section 4 footnote / Lemma 3 /
 * Section 5 widths).  host_T[r], host_alpha[r] for r < *R (cumulative
 * sample targets of the sampled rounds); round *R is the exact round.
 * Arrays must hold KNN_MAX_ROUNDS entries.  Host only. */
int knn_schedule(const knn_params *p, int64_t n, int64_t m, int32_t *host_T,
                 double *host_alpha, int32_t *R);

/* Adaptive k-NN (Algorithm 1, round-synchronous form) for nq queries.
 *  dev_queries : device, [nq][m], same dtype as the DB.
 *  host_k      : host, [nq], k_q >= 1.
 *  p, np       : host parameter array of length np = 1 (shared) or nq.
 *  dev_out_idx : device, [nq][out_stride] int64; row q receives the returned
 *                set (at most k_q + h_q indices, ordered by estimate then index),
 *                padded with -1.  out_stride >= max_q (k_q + h_q).
 *  dev_out_count: device, [nq] int32, returned set sizes.
 *  dev_out_stats: device, [nq] knn_stats, or NULL.
 * With probability >= 1 - delta (per query) the set contains the k nearest
 * neighbours (Theorem 1).  If k_q + h_q >= n all n points are returned.
 * Stream-ordered on `stream`; may synchronise it when the queries do not
 * all fit in device memory at once.  Errors: EINVAL (k < 1, k+h > KNN_MAX_KH,
 * delta outside (0,1), b0 not a positive multiple of 4, growth < 1, schedule
 * longer than KNN_MAX_ROUNDS, c_exact < 0, alpha_kind 2 with c_alpha <= 0,
 * NULL pointers, out_stride too small), ENOMEM, EDEVICE. */
int knn_adaptive(knn_db db, const void *dev_queries, int64_t nq, const int32_t *host_k,
                 const knn_params *p, int64_t np, int64_t *dev_out_idx, int64_t out_stride,
                 int32_t *dev_out_count, knn_stats *dev_out_stats, void *stream);

/* Debug/parity hook: runs the same call as knn_adaptive (same arguments:
 * nq queries, host_k[nq], p[np]) with every query in flight at once, stops
 * each query after `stop_after` decide steps, and copies the per-point state
 * of query `query` to host arrays of length n: S (int64 running sums), fl
 * (bit 0 exact, bit 1 accepted, bit 2 discarded) and ri (round index of the
 * point's last sampled target).  A query that finished in fewer decide steps
 * leaves its final state.  The batch takes the launch path knn_adaptive
 * would take for it (shared-seed batches: the query-lane kernels and their
 * point-major sums), so the state of any slot of such a batch can be
 * compared with a reference run of that query alone.  Synchronous.
 * Errors: EINVAL (as knn_adaptive, stop_after < 1, query outside [0, nq),
 * a trivial query), ENOMEM (the nq queries do not fit in device memory at
 * once), EDEVICE. */
int knn_adaptive_state(knn_db db, const void *dev_queries, int64_t nq, const int32_t *host_k,
                       const knn_params *p, int64_t np, int64_t query, int32_t stop_after,
                       int64_t *host_S, uint8_t *host_fl, uint8_t *host_ri, void *stream);

/* Autotuner for the performance knobs of the adaptive path (none of them
 * changes a result): runs knn_adaptive on these queries (same k for all,
 * params shared) once per candidate -- query-lane vs grouped vs per-query
 * sampling, points per sampling block, lanes per point, graph replay --
 * times each on `stream` with HIP events (one untimed warm-up, then the
 * mean of `reps` runs), checks that every candidate returns the same
 * indices, counts and statistics as the first, and keeps the fastest for
 * this DB (used by later calls; KNN_* environment variables still
 * override).  The result-defining schedule (B0, growth g of the round
 * targets, Section 4) is never changed; when `schedule_report` is nonzero
 * the times of B0 in {16, 64, 256} x g in {1.5, 2} are measured and
 * reported too, as a recommendation only.
 *  report: host buffer (nullable) receiving one line per measurement,
 *          "name ms" (truncated to report_len, NUL-terminated).
 * Synchronous; not to be called concurrently with other calls on the same
 * DB.  Errors: EINVAL, ENOMEM, EDEVICE (also when a candidate's output
 * differs from the first one's). */
int knn_autotune(knn_db db, const void *dev_queries, int64_t nq, int32_t k, const knn_params *p,
                 int32_t reps, int32_t schedule_report, char *report, size_t report_len, void *stream);

/* ------------------------------------------------------------- naive --- */

/* Naive k-NN (Section 3): all n distances, the k smallest by (distance,
 * index).  Squared l2 -- u8: exact integer distances via int8 MFMA; f32:
 * BF16 MFMA candidates, rescored in FP64 in coordinate order, so the set and
 * the distances equal an FP64 scan.  l1 (no matrix-core form) -- u8: exact
 * integer sums of absolute differences (v_sad_u8); f32: fp32 sums with an
 * error bound, candidates rescored in FP64 in coordinate order.
 * Above the fused top-k lists' capacity (u8 k > 128, f32 k > 64) every query
 * is scanned exactly instead, one block per query with the k smallest found
 * by radix selection over all n keys (integer distances for u8, FP64 in
 * coordinate order for f32): the same results, at a DB read per query.
 *  dev_out_idx : device, [nq][k] int64 (ascending distance).
 *  dev_out_dist: device, [nq][k] double (unnormalised squared l2 or l1
 *                distance), or NULL.
 * Stream-ordered (the f32 exact scans synchronise the stream before
 * returning).  Errors: EINVAL (k < 1, k > min(n, KNN_MAX_KH), NULL), ENOMEM,
 * EDEVICE. */
int knn_naive(knn_db db, const void *dev_queries, int64_t nq, int32_t k,
              int64_t *dev_out_idx, double *dev_out_dist, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, serving loops and harnesses that forbid allocation: knn_naive on
 * a u8 DB (same arguments, same results) that calls no allocator.  Its
 * working memory (the shifted query rows, nq * (mp + 4) + 512 bytes with mp
 * = m rounded up to 64, and 8 * k bytes per query and point range for the
 * candidate lists) lives in a fixed array of KNN_NOALLOC_SCRATCH_MB MiB that
 * the library holds on each device it runs on until the process ends; the
 * point ranges are widened until the lists fit.  Every call on a device
 * shares that device's array: calls that overlap on one GPU (on different
 * streams, or from several threads) race -- serialise them.  Nothing in the
 * array needs clearing between calls.  Stream-ordered.  Errors: as
 * knn_naive, plus EINVAL for an f32 DB, for k > 128 (the exact per-query
 * scan needs scratch of 8 n bytes per query) and for a batch whose query
 * rows alone do not fit (the message gives the bytes needed). */
#define KNN_NOALLOC_SCRATCH_MB 64
int knn_naive_noalloc(knn_db db, const void *dev_queries, int64_t nq, int32_t k,
                      int64_t *dev_out_idx, double *dev_out_dist, void *stream);

/* ----------------------------------------------------------- session --- */

/* Serving session: resident DBs, a background loop per DB that admits
 * submitted queries while their state fits hbm_budget_bytes, and runs
 * admitted queries of different k and delta together (continuous batching:
 * queries join at round boundaries of queries already running).  The budget
 * is shared by all DBs: an admitted query holds its DB's per-query state
 * (about 34 bytes per point of the DB, plus its result row) until its result
 * has been copied out.  Each DB's slot arena is sized so that the DB alone
 * can use the whole budget (at most 1024 queries in flight per DB).
 * Errors: EINVAL (budget below 1 MiB, NULL). */
int knn_session_create(size_t hbm_budget_bytes, knn_session *out);

/* Makes `db` resident in the session; *db_id identifies it in submit.
 * Errors: EINVAL, ENOMEM (the budget does not hold one query of this DB, or
 * the slot arena cannot be allocated), EDEVICE. */
int knn_session_add_db(knn_session s, knn_db db, int32_t *db_id);

/* Enqueues one query (host_query: host, [m] of the DB's dtype; copied
 * before return).  Never blocks on the GPU.  *ticket identifies the
 * request.  Errors: EINVAL, ENOTFOUND (db_id). */
int knn_session_submit(knn_session s, int32_t db_id, const void *host_query, int32_t k,
                       const knn_params *p, uint64_t *ticket);

/* KNN_PENDING until the request is done; then copies its result
 * (host_idx: at least k+h entries, -1 padded), frees the ticket and
 * returns KNN_OK.  ENOTFOUND for unknown tickets. */
int knn_session_poll(knn_session s, uint64_t ticket, int64_t *host_idx, int32_t *count,
                     knn_stats *st);

/* Stops the loop, waits for in-flight work, frees session memory. */
int knn_session_destroy(knn_session s);

/* ------------------------------------------------------- measurement --- */

/* Kernel timing for benchmarks.  knn_prof_enable(1) clears the records and
 * turns timing on: every launch of a hot kernel class is then bracketed by
 * HIP events on the stream it is launched on, and the adaptive sampling
 * kernel adds its algorithmic work to device counters.  Off by default
 * (no events, no counters).  knn_prof_enable(0) turns it off. */
int knn_prof_enable(int on);

/* Total event time (ms), launch count and algorithmic work units of one
 * kernel class since the last enable: 0 adaptive sampling (units: bytes),
 * 1 candidate-exact, 2 bound selection, 3 decide/compact, 4 finish/admit,
 * 5 naive MFMA scan (units: integer or floating-point operations, 2 per
 * multiply-add), 6 naive query prep / merge / rescoring, 7 adaptive sampling
 * launches that run the exact round of a batch whose queries all share one
 * schedule (such launches are counted here instead of under 0), 8 the
 * point-major / slot-major transposes around query-lane sampling (flags in,
 * round totals out; under 0 is then the sampling kernel alone), or the
 * gather of the points and queries at a shared coordinate sequence, 9 the
 * per-query sampling (or exact sums) of the queries of a point-major batch
 * whose undecided sets have become small.  Waits for the recorded events. */
int knn_prof_read(int32_t kind, double *total_ms, int64_t *launches, double *units);

/* Work counters since the last enable: [0] algorithmic bytes of the
 * adaptive sampling kernel, [1] (query, sample) pairs drawn, [2] exact-distance
 * (query, coordinate) pairs, [3] distinct coordinate draws (queries sharing a
 * seed share them), [4] float naive queries that fell back to an exact rescan,
 * [5] distinct draws of shared coordinate sequences (one sequence serves a
 * whole batch), [6..7] reserved.  host_out8: host, 8 entries.  Synchronises the device. */
int knn_prof_counters(uint64_t *host_out8);

#ifdef __cplusplus
}
#endif
#endif
