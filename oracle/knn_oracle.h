/*
 * knn_oracle.h -- plain, slow, single-threaded CPU oracle for adaptive
 * k-NN (LeJeune, Baraniuk, Heckel, "Adaptive Estimation for Approximate
 * k-Nearest-Neighbor Computations", AISTATS 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * library (libknn) never links, loads or calls it, and it shares no code
 * with the product: its own Philox, its own confidence bounds, its own
 * schedule, its own selection, all written from the paper.
 *
 * Precision: integer sums in int64, every bound in IEEE double with no
 * fused multiply-add (built with -ffp-contract=off), natural logarithms.
 */
#ifndef KNN_ORACLE_H
#define KNN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_U8 = 0, ORC_F32 = 1 };
/* Distance: squared l2 (the paper's), or l1 (Section 3: the results carry
 * over to it), whose samples are |x_ij - x_j| instead of (x_ij - x_j)^2. */
enum { ORC_L2 = 0, ORC_L1 = 1 };

/* Result-defining parameters of one query (same field order and meaning as
 * the product's parameter struct, so one Python object can fill both). */
typedef struct {
  int64_t  h;           /* slack; < 0 means h = k */
  double   delta;       /* failure probability, (0,1) */
  uint64_t seed;        /* Philox key */
  int32_t  alpha_kind;  /* 0 footnote beta, 1 Lemma-3 beta, 2 experimental C_alpha */
  double   c_alpha;     /* only for alpha_kind 2 */
  int32_t  b0;          /* samples per point in round 0 (multiple of 4); 0 -> 64 */
  float    growth;      /* T grows by max(4, ceil4(T*(g-1))) per round; 0 -> 2 */
  float    theta_exact; /* go exact once the next target reaches ceil(theta*m); 0 -> 1 */
  int32_t  c_exact;     /* candidate-exact count (0 = pure round form) */
  int32_t  sampling;    /* coordinates of point i: 0 drawn with replacement (orc_index),
                            1 without (orc_perm_index); one sequence shared by all points:
                            2 with replacement (orc_shared_index), 3 without
                            (orc_shared_perm_index) */
} orc_params;

typedef struct {
  int64_t coord_evals;  /* coordinate evaluations: samples + m per exact point */
  int32_t rounds;       /* decide steps executed */
  int32_t count;        /* returned set size */
  int64_t exact_points; /* points whose distance was computed exactly */
} orc_stats;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
 * Philox S-box keyed by a Weyl sequence. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Raw 32-bit draw for sample t of point i under seed: output t mod 4 of
 * Philox4x32-10 with key = (seed lo, seed hi), counter = (t/4, 0, i, 0). */
uint32_t orc_draw(uint64_t seed, int64_t i, int64_t t);

/* Coordinate index of that sample: floor(draw * m / 2^32). */
int64_t orc_index(uint64_t seed, int64_t i, int64_t t, int64_t m);

/* Confidence width alpha(u) of Section 4 (footnote form, kind 0), of
 * Lemma 3 (kind 1) or of the experiments section (kind 2). Kind 0 falls
 * back to kind 1 when delta/n >= 0.05.  Returns NaN on invalid input. */
double orc_alpha(int32_t kind, int64_t u, int64_t n, double delta, double c_alpha);

/* Sampling without replacement (Section 4 footnote): sample t (< m) of
 * point i is pi(t), pi a permutation of [0, m): a four-round Feistel
 * network on 2h bits, h = max(1, ceil(ceil(log2 m) / 2)), halves of h
 * bits, (L, R) -> (R, L xor F(k_r, R)) with F(k, v) = lowbias32(v xor k)
 * mod 2^h, round keys k_0..k_3 = Philox4x32-10(key = seed, counter =
 * (0, 0, i, 1)); values >= m are enciphered again until they fall in
 * [0, m) (cycle walking, Black & Rogaway 2002).  lowbias32(x): x ^= x >> 16;
 * x *= 0x7feb352d; x ^= x >> 15; x *= 0x846ca68b; x ^= x >> 16. */
int64_t orc_perm_index(uint64_t seed, int64_t i, int64_t t, int64_t m);

/* One coordinate sequence for all points (Section 4 writes every point's
 * estimator over the same j_1, j_2, ...): the 32-bit draw of sample t
 * (Philox counter (t/4, 0, 0, 2)), its coordinate, the coordinate without
 * replacement (round keys from counter (0, 0, 0, 3)), and the coordinate of
 * sample t of point i under any sampling mode 0..3. */
uint32_t orc_draw_shared(uint64_t seed, int64_t t);
int64_t orc_shared_index(uint64_t seed, int64_t t, int64_t m);
int64_t orc_shared_perm_index(uint64_t seed, int64_t t, int64_t m);
int64_t orc_coord(int32_t sampling, uint64_t seed, int64_t i, int64_t t, int64_t m);

/* Round schedule: fills T[0..R-1] with the cumulative sample targets of the
 * sampled rounds; round R is the exact round.  Returns R, or -1 if the
 * schedule would exceed maxlen rounds or the parameters are invalid. */
int32_t orc_schedule(int32_t b0, float growth, float theta, int64_t m,
                     int32_t *T, int32_t maxlen);

/* Fixed-point scaling for float data: W (samples s/W lie in [0,1]) and the
 * shift F; for u8 W = 255^2 (l1: 255) and F = 0.  For f32, with R = hi - lo
 * over the points and the query, R' = R^2 (1 + 2^-20) (l1: R (1 + 2^-20)),
 * F = 61 - ceil(log2 m) - ceil(log2 R') and W = R' 2^F.  Returns 0 ok,
 * 1 degenerate (zero range), <0 invalid. */
int32_t orc_scaling(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                    const void *q, double *W, int32_t *F);

/* Adaptive k-NN, round-synchronous form of Algorithm 1.
 * out_idx: [k+h] (padded with -1).  stop_after > 0 stops after that many
 * decide steps without finalising (for state comparison); the per-point
 * state is then written to S_dump / fl_dump / ri_dump when non-NULL.
 * Returns 0 ok, <0 invalid arguments. */
int32_t orc_adaptive(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                     const void *q, int32_t k, const orc_params *p,
                     int32_t stop_after, int64_t *out_idx, orc_stats *st,
                     int64_t *S_dump, uint8_t *fl_dump, uint8_t *ri_dump);

/* Algorithm 1 exactly as published (Section 4): sequential LUCB.  One
 * sample per point to start; then, per iteration, with the points ordered
 * by (d^, index): q1 = argmax of d^ + alpha over the first k, q2 = argmin
 * of d^ - alpha over positions k+h+1..n, b2 = argmax of alpha over q2 and
 * positions k+1..k+h (eq. d_ind, eq. blowbupdef; ties to the first listed,
 * then the smaller index).  Stops when d^_q1 + alpha_q1 <= d^_q2 - alpha_q2
 * (eq. termination); otherwise q1 and b2 take one more sample each; a point
 * whose count reaches ceil(theta m) gets its exact distance and alpha = 0.
 * The t-th sample of point i uses the same Philox draw as the round form.
 * out_idx: [k+h], the first k+h by (d^, index).  st: coord_evals (samples
 * + m per exact point), rounds = iterations, count, exact_points.
 * T_out (nullable): [n] final sample counts.  Returns 0 ok, -1 invalid
 * arguments, -2 when max_iter iterations did not terminate. */
int32_t orc_alg1(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                 const void *q, int32_t k, const orc_params *p, int64_t max_iter,
                 int64_t *out_idx, orc_stats *st, int64_t *T_out);

/* Algorithm 1 with the bookkeeping of Section 4.1 (Figure fig:heaps): the
 * first k, the next h and the remaining points by (d^, index) each keep
 * coupled binary heaps (close: max on d^ and on d^ + alpha; middle: min and
 * max on d^, max on alpha; far: min on d^ and on d^ - alpha), built bottom-up
 * (Floyd); q1, q2 and b2 are heap tops, and after an iteration's updates
 * extreme points are swapped between neighbouring sets until the order
 * holds again -- O(log n) per iteration.  Same arguments, ties and results
 * as orc_alg1. */
int32_t orc_alg1_heaps(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                       const void *q, int32_t k, const orc_params *p, int64_t max_iter,
                       int64_t *out_idx, orc_stats *st, int64_t *T_out);

/* Naive brute force of Section 3: all distances, k smallest by (d, index).
 * u8: exact int64 sums; f32: double sums in coordinate order.
 * out_dist receives the unnormalised distances (squared l2, or l1). */
int32_t orc_naive(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                  const void *q, int32_t k, int64_t *out_idx, double *out_dist);

/* Exact distance of one point (unnormalised squared l2, or l1), as the
 * naive scan computes it. */
double orc_exact_dist(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                      const void *q, int64_t i);

#ifdef __cplusplus
}
#endif
#endif
