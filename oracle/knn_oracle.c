/*
 * knn_oracle.c -- plain CPU oracle for adaptive k-NN.  TEST INFRASTRUCTURE
 * ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg
 * are its only users; the product library never touches it.
 *
 * Paper: LeJeune, Baraniuk, Heckel, "Adaptive Estimation for Approximate
 * k-Nearest-Neighbor Computations" (AISTATS 2019).  Every function below
 * names the passage it follows.  It is written for a reader checking it
 * against the paper: no blocking, no fusion, sorts where the paper sorts.
 *
 * Round-synchronous reading of Algorithm 1 (the paper gives only the
 * one-sample-per-iteration form): every undecided point is sampled each
 * round up to a common target T_r; then, on one snapshot of the bounds,
 *   U  = k-th smallest upper bound (d^ + alpha) over the kept set P,
 *   L1 = k-th, L2 = (k+1)-th smallest lower bound (d^ - alpha) over P,
 * an undecided point is discarded when its lower bound exceeds U (k kept
 * points are then surely closer) and accepted when fewer than k other
 * points can be closer (upper bound <= L2, or for an exact point d <= L1).
 * Lemma 3's event holds for all points and all sample counts at once, so
 * any such schedule keeps the k nearest neighbours with probability
 * >= 1 - delta.  The run stops once |P| <= k+h or no undecided point is
 * left to sample.
 */
#include "knn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as  */
/* 1, 2, 3", SC'11): multipliers and Weyl key increments as published. */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint32_t orc_draw(uint64_t seed, int64_t i, int64_t t) {
  uint32_t ctr[4] = {(uint32_t)(t / 4), 0u, (uint32_t)i, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[t % 4];
}

/* Section 4: indices are drawn uniformly from [m]; a 32-bit draw r maps to
 * floor(r*m/2^32) (bias at most m/2^32 per index, none when m is a power
 * of two). */
int64_t orc_index(uint64_t seed, int64_t i, int64_t t, int64_t m) {
  uint64_t r = orc_draw(seed, i, t);
  return (int64_t)((r * (uint64_t)m) >> 32);
}

/* ------------------------------------------------------------------ */
/* Confidence widths.                                                   */
/* ------------------------------------------------------------------ */

/* Section 4, footnote to the definition of alpha: the non-asymptotic law
 * of the iterated logarithm,
 *   beta(u, d') = log(1/d') + 3 log log(1/d') + 1.5 log(1 + log u),
 *   alpha(u)    = sqrt(2 beta(u, delta/n) / u). */
static double beta_footnote(double u, double dp) {
  double l = log(1.0 / dp);
  return l + 3.0 * log(l) + 1.5 * log(1.0 + log(u));
}

/* Section 6, Lemma 3 (second statement, valid for every delta in (0,1)):
 *   beta(t, d') = 2 log(125 log(1.12 t) / d'). */
static double beta_lemma(double t, double dp) {
  return 2.0 * log(125.0 * log(1.12 * t) / dp);
}

double orc_alpha(int32_t kind, int64_t u, int64_t n, double delta, double c_alpha) {
  if (u < 1 || n < 1 || !(delta > 0.0 && delta < 1.0)) return NAN;
  double du = (double)u;
  if (kind == 2) {
    /* Section 5 (experiments): alpha(u) = sqrt(C log(1 + (1 + log u) n / delta) / u). */
    if (!(c_alpha > 0.0)) return NAN;
    return sqrt(c_alpha * log(1.0 + (1.0 + log(du)) * (double)n / delta) / du);
  }
  double dp = delta / (double)n;
  double b;
  if (kind == 0 && dp < 0.05) b = beta_footnote(du, dp);
  else if (kind == 0 || kind == 1) b = beta_lemma(du, dp);
  else return NAN;
  return sqrt(2.0 * b / du);
}

/* ------------------------------------------------------------------ */
/* Sampling without replacement: a keyed permutation of [0, m) (Section  */
/* 4 footnote; Black & Rogaway's cycle-walking cipher on a Feistel       */
/* network).                                                             */
/* ------------------------------------------------------------------ */
static uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

/* Position t < m of the permutation whose four Feistel round keys are the
 * Philox outputs for counter (0, 0, c2, c3). */
static int64_t perm_at(uint64_t seed, uint32_t c2, uint32_t c3, int64_t t, int64_t m) {
  uint32_t ctr[4] = {0u, 0u, c2, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t rk[4];
  orc_philox4x32_10(ctr, key, rk);
  int bits = 0;
  while (((int64_t)1 << bits) < m) ++bits;  /* ceil(log2 m) */
  int h = (bits + 1) / 2;
  if (h < 1) h = 1;
  const uint32_t mask = (h >= 32) ? 0xFFFFFFFFu : ((1u << h) - 1u);
  uint64_t x = (uint64_t)t;
  do {
    uint32_t L = (uint32_t)(x >> h) & mask, R = (uint32_t)x & mask;
    for (int r = 0; r < 4; ++r) {
      const uint32_t nr = L ^ (lowbias32(R ^ rk[r]) & mask);
      L = R;
      R = nr;
    }
    x = ((uint64_t)L << h) | R;
  } while ((int64_t)x >= m);
  return (int64_t)x;
}

/* Per-point permutation: round keys from counter (0, 0, i, 1). */
int64_t orc_perm_index(uint64_t seed, int64_t i, int64_t t, int64_t m) {
  return perm_at(seed, (uint32_t)i, 1u, t, m);
}

/* ------------------------------------------------------------------ */
/* One coordinate sequence for all points.  Section 4 writes the        */
/* estimator of every point with the same indices j_1, j_2, ...; point i */
/* uses the first T_i of them.  Lemma 3 needs, per point, i.i.d. samples */
/* that are bounded and unbiased; it says nothing about how the samples  */
/* of different points relate (its event is a union over points), so a   */
/* sequence shared by all points keeps the guarantee.                    */
/*   with replacement:    j_t = floor(r m / 2^32), r = output (t mod 4)  */
/*                        of Philox4x32-10(seed, counter (t/4, 0, 0, 2));*/
/*   without replacement: j_t = pi(t), pi the Feistel permutation above  */
/*                        with round keys from counter (0, 0, 0, 3).     */
/* ------------------------------------------------------------------ */
uint32_t orc_draw_shared(uint64_t seed, int64_t t) {
  uint32_t ctr[4] = {(uint32_t)(t / 4), 0u, 0u, 2u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[t % 4];
}

int64_t orc_shared_index(uint64_t seed, int64_t t, int64_t m) {
  uint64_t r = orc_draw_shared(seed, t);
  return (int64_t)((r * (uint64_t)m) >> 32);
}

int64_t orc_shared_perm_index(uint64_t seed, int64_t t, int64_t m) {
  return perm_at(seed, 0u, 3u, t, m);
}

/* Coordinate of sample t of point i under sampling mode 0 (per point, with
 * replacement), 1 (per point, without), 2 (shared, with), 3 (shared,
 * without). */
int64_t orc_coord(int32_t sampling, uint64_t seed, int64_t i, int64_t t, int64_t m) {
  switch (sampling) {
    case 1: return orc_perm_index(seed, i, t, m);
    case 2: return orc_shared_index(seed, t, m);
    case 3: return orc_shared_perm_index(seed, t, m);
    default: return orc_index(seed, i, t, m);
  }
}

/* ------------------------------------------------------------------ */
/* Round schedule (round-synchronous reading; Algorithm 1 takes one     */
/* sample per iteration, here a round takes B samples per point).      */
/* ------------------------------------------------------------------ */
int32_t orc_schedule(int32_t b0, float growth, float theta, int64_t m,
                     int32_t *T, int32_t maxlen) {
  if (b0 == 0) b0 = 64;
  if (growth == 0.0f) growth = 2.0f;
  if (theta == 0.0f) theta = 1.0f;
  if (b0 < 4 || (b0 % 4) != 0 || !(growth >= 1.0f) || !(theta > 0.0f) || m < 1) return -1;
  /* exact threshold: ceil(theta * m), clipped to [1, m] (Algorithm 1: a
   * point whose count reaches m gets its exact distance). */
  double thr_d = ceil((double)theta * (double)m);
  int64_t thr = thr_d >= (double)m ? m : (int64_t)thr_d;
  if (thr < 1) thr = 1;
  int32_t R = 0;
  int64_t t = b0;
  while (t < thr) {
    if (R >= maxlen) return -1;
    T[R++] = (int32_t)t;
    double g1 = (double)t * ((double)growth - 1.0);
    int64_t b = (int64_t)ceil(g1);
    b = ((b + 3) / 4) * 4;
    if (b < 4) b = 4;
    t += b;
  }
  return R;
}

/* ------------------------------------------------------------------ */
/* Sample values.  Section 3 asks for coordinates with |x_j| <= 1/2 so   */
/* that every sample |x_ij - x_j|^2 lies in [0,1]; Lemma 3 needs exactly */
/* that.  Here samples are kept as integers and divided by W:           */
/*   u8:  s = (x_ij - x_j)^2,            W = 255^2;                      */
/*   f32: s = trunc(fl32(fl32(x_ij - x_j)^2) * 2^F),  W = R' 2^F, where  */
/*        R' = (hi - lo)^2 (1 + 2^-20) over the points and the query.    */
/* The l1 distance (Section 3 remarks that the results carry over to it)  */
/* samples |x_ij - x_j| instead, which lies in [0,1] under the same      */
/* normalisation, so the same estimator and widths apply:                */
/*   u8:  s = |x_ij - x_j|,              W = 255;                        */
/*   f32: s = trunc(|fl32(x_ij - x_j)| * 2^F),  W = R' 2^F with          */
/*        R' = (hi - lo) (1 + 2^-20).                                    */
/* ------------------------------------------------------------------ */
typedef struct {
  const uint8_t *xu;
  const float *xf;
  const uint8_t *qu;
  const float *qf;
  int64_t n, m;
  int32_t dtype;
  int32_t metric; /* ORC_L2 or ORC_L1 */
  double W;
  double scale; /* 2^F */
  int32_t sampling; /* 0..3, see orc_coord */
  int32_t norepl;   /* sampling without replacement (modes 1 and 3) */
} inst_t;

static int ceil_log2(double x) {
  int e;
  double f = frexp(x, &e); /* x = f 2^e, f in [0.5, 1) */
  return (f == 0.5) ? e - 1 : e;
}

int32_t orc_scaling(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                    const void *q, double *W, int32_t *F) {
  if (metric != ORC_L2 && metric != ORC_L1) return -1;
  if (dtype == ORC_U8) { *W = metric == ORC_L1 ? 255.0 : 65025.0; *F = 0; return 0; }
  if (dtype != ORC_F32) return -1;
  const float *xf = (const float *)X, *qf = (const float *)q;
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t a = 0; a < n * m; ++a) {
    double v = (double)xf[a];
    if (v < lo) lo = v;
    if (v > hi) hi = v;
  }
  for (int64_t j = 0; j < m; ++j) {
    double v = (double)qf[j];
    if (v < lo) lo = v;
    if (v > hi) hi = v;
  }
  double span = hi - lo;
  if (!(span > 0.0)) { *W = 0.0; *F = 0; return 1; }
  double Rp = (metric == ORC_L1 ? span : span * span) * (1.0 + 0x1p-20);
  int f = 61 - ceil_log2((double)m) - ceil_log2(Rp);
  *F = f;
  *W = ldexp(Rp, f);
  return 0;
}

static int64_t sample_value(const inst_t *I, int64_t i, int64_t j) {
  if (I->dtype == ORC_U8) {
    int64_t d = (int64_t)I->xu[i * I->m + j] - (int64_t)I->qu[j];
    if (I->metric == ORC_L1) return d < 0 ? -d : d;
    return d * d;
  }
  float d = I->xf[i * I->m + j] - I->qf[j];
  float v = I->metric == ORC_L1 ? fabsf(d) : d * d;
  return (int64_t)((double)v * I->scale);
}

/* Algorithm 1: "compute the distance exactly" -- all m coordinates. */
static int64_t exact_sum(const inst_t *I, int64_t i) {
  int64_t s = 0;
  for (int64_t j = 0; j < I->m; ++j) s += sample_value(I, i, j);
  return s;
}

/* Section 4 estimator: sum of samples t0..t1-1 of point i. */
static int64_t sampled_sum(const inst_t *I, uint64_t seed, int64_t i, int64_t t0, int64_t t1) {
  int64_t s = 0;
  for (int64_t t = t0; t < t1; ++t)
    s += sample_value(I, i, orc_coord(I->sampling, seed, i, t, I->m));
  return s;
}

/* Coordinates an exact distance costs on top of T samples already drawn:
 * all m with replacement, the m - T not yet seen without. */
static int64_t exact_cost(const inst_t *I, int64_t T) {
  return I->norepl ? I->m - T : I->m;
}

/* d^_i(T) = S / (T W): the Section 4 estimate in the [0,1] normalisation. */
static double dhat_of(const inst_t *I, int64_t S, int64_t T) {
  return (double)S / ((double)T * I->W);
}

/* ------------------------------------------------------------------ */
/* Sorting helpers (plain qsort).                                       */
/* ------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x < y) ? -1 : (x > y) ? 1 : 0;
}

typedef struct { double key; int64_t idx; } keyidx_t;

static int cmp_keyidx(const void *a, const void *b) {
  const keyidx_t *x = (const keyidx_t *)a, *y = (const keyidx_t *)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->idx < y->idx) ? -1 : (x->idx > y->idx) ? 1 : 0;
}

/* r-th smallest (1-based) of v[0..len-1]; sorts v. */
static double kth_smallest(double *v, int64_t len, int64_t r) {
  qsort(v, (size_t)len, sizeof(double), cmp_double);
  return v[r - 1];
}

/* ------------------------------------------------------------------ */
/* Adaptive k-NN.                                                       */
/* ------------------------------------------------------------------ */
#define FL_EXACT 1u
#define FL_ACC 2u
#define FL_DISC 4u
#define MAX_ROUNDS 64

int32_t orc_adaptive(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                     const void *q, int32_t k, const orc_params *p,
                     int32_t stop_after, int64_t *out_idx, orc_stats *st,
                     int64_t *S_dump, uint8_t *fl_dump, uint8_t *ri_dump) {
  if (!X || !q || !p || !out_idx || !st || n < 1 || m < 1 || k < 1) return -1;
  if (dtype != ORC_U8 && dtype != ORC_F32) return -1;
  if (!(p->delta > 0.0 && p->delta < 1.0)) return -1;
  int64_t h = p->h < 0 ? (int64_t)k : p->h;
  int64_t kh = (int64_t)k + h;
  int32_t T[MAX_ROUNDS];
  int32_t R = orc_schedule(p->b0, p->growth, p->theta_exact, m, T, MAX_ROUNDS);
  if (R < 0) return -1;
  if (p->c_exact < 0) return -1;
  if (p->alpha_kind < 0 || p->alpha_kind > 2) return -1;
  if (p->alpha_kind == 2 && !(p->c_alpha > 0.0)) return -1;
  memset(st, 0, sizeof(*st));
  for (int64_t a = 0; a < kh; ++a) out_idx[a] = -1;

  /* Section 3: with n <= k+h every point belongs to the answer. */
  if (n <= kh) {
    for (int64_t i = 0; i < n; ++i) out_idx[i] = i;
    st->count = (int32_t)n;
    return 0;
  }

  inst_t I;
  memset(&I, 0, sizeof(I));
  I.n = n; I.m = m; I.dtype = dtype; I.metric = metric;
  if (dtype == ORC_U8) { I.xu = (const uint8_t *)X; I.qu = (const uint8_t *)q; }
  else { I.xf = (const float *)X; I.qf = (const float *)q; }
  int32_t F;
  int32_t sc = orc_scaling(X, n, m, dtype, metric, q, &I.W, &F);
  if (sc < 0) return -1;
  if (sc == 1) {
    /* zero range: every distance is 0, any k+h points are an answer */
    for (int64_t a = 0; a < kh; ++a) out_idx[a] = a;
    st->count = (int32_t)kh;
    return 0;
  }
  I.scale = ldexp(1.0, F);
  if (p->sampling < 0 || p->sampling > 3) return -1;
  I.sampling = p->sampling;
  I.norepl = p->sampling & 1;

  double alpha_r[MAX_ROUNDS];
  for (int32_t r = 0; r < R; ++r) {
    alpha_r[r] = orc_alpha(p->alpha_kind, T[r], n, p->delta, p->c_alpha);
    if (!(alpha_r[r] >= 0.0)) return -1;
  }

  int64_t *S = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  uint8_t *fl = (uint8_t *)calloc((size_t)n, 1);
  uint8_t *ri = (uint8_t *)calloc((size_t)n, 1);
  double *ucb = (double *)malloc((size_t)n * sizeof(double));
  double *lcb = (double *)malloc((size_t)n * sizeof(double));
  double *tmp = (double *)malloc((size_t)n * sizeof(double));
  keyidx_t *ki = (keyidx_t *)malloc((size_t)n * sizeof(keyidx_t));
  if (!S || !fl || !ri || !ucb || !lcb || !tmp || !ki) {
    free(S); free(fl); free(ri); free(ucb); free(lcb); free(tmp); free(ki);
    return -2;
  }

  /* Algorithm 1 initialisation: every point gets its first samples (B0 of
   * them here), or its exact distance when B0 already reaches the exact
   * threshold. */
  int32_t cur = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (R == 0) {
      S[i] = exact_sum(&I, i);
      fl[i] = FL_EXACT;
      st->coord_evals += m;
      st->exact_points += 1;
    } else {
      S[i] = sampled_sum(&I, p->seed, i, 0, T[0]);
      ri[i] = 0;
      st->coord_evals += T[0];
    }
  }

  int finished = 0;
  for (;;) {
    st->rounds += 1;

    /* Candidate-exact (optional): the c_exact undecided points with the
     * smallest estimate (ties by index) get exact distances. */
    if (p->c_exact > 0) {
      int64_t na = 0;
      for (int64_t i = 0; i < n; ++i) {
        if (fl[i] & (FL_ACC | FL_DISC)) continue;
        int64_t Tn = (fl[i] & FL_EXACT) ? m : T[ri[i]];
        ki[na].key = dhat_of(&I, S[i], Tn);
        ki[na].idx = i;
        ++na;
      }
      qsort(ki, (size_t)na, sizeof(keyidx_t), cmp_keyidx);
      int64_t c = p->c_exact < na ? p->c_exact : na;
      for (int64_t a = 0; a < c; ++a) {
        int64_t i = ki[a].idx;
        if (fl[i] & FL_EXACT) continue;
        S[i] = exact_sum(&I, i);
        fl[i] |= FL_EXACT;
        st->coord_evals += exact_cost(&I, T[ri[i]]);
        st->exact_points += 1;
      }
    }

    /* Bounds on P (everything not discarded): d^ +- alpha(T), alpha = 0
     * for exact points (Algorithm 1). */
    int64_t np = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (fl[i] & FL_DISC) continue;
      double d, a;
      if (fl[i] & FL_EXACT) { d = dhat_of(&I, S[i], m); a = 0.0; }
      else { d = dhat_of(&I, S[i], T[ri[i]]); a = alpha_r[ri[i]]; }
      ucb[i] = d + a;
      lcb[i] = d - a;
      tmp[np++] = ucb[i];
    }
    /* Equation (d_ind) picks the worst of the k apparently closest points;
     * in round form the k-th smallest upper bound plays that role. */
    double U = kth_smallest(tmp, np, k);
    int64_t nl = 0;
    for (int64_t i = 0; i < n; ++i)
      if (!(fl[i] & FL_DISC)) tmp[nl++] = lcb[i];
    qsort(tmp, (size_t)nl, sizeof(double), cmp_double);
    double L1 = tmp[k - 1];
    double L2 = tmp[k];

    /* Decide, all undecided points at once on this snapshot. */
    int64_t n_act = 0, n_p = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (fl[i] & (FL_ACC | FL_DISC)) continue;
      int exact = (fl[i] & FL_EXACT) != 0;
      if (lcb[i] > U) {
        fl[i] |= FL_DISC;
      } else if ((!exact && ucb[i] <= L2) || (exact && ucb[i] <= L1)) {
        fl[i] |= FL_ACC;
      }
    }
    for (int64_t i = 0; i < n; ++i) {
      if (fl[i] & FL_DISC) continue;
      ++n_p;
      if (!(fl[i] & (FL_ACC | FL_EXACT))) ++n_act;
    }

    if (stop_after > 0 && st->rounds >= stop_after) break;

    /* Stop once the kept set is small enough (the size bound of Theorem 1)
     * or nothing is left to sample. */
    if (n_p <= kh || n_act == 0) { finished = 1; break; }

    /* Next round: sample the undecided, or compute them exactly once the
     * next target reaches the exact threshold. */
    ++cur;
    for (int64_t i = 0; i < n; ++i) {
      if (fl[i] & (FL_ACC | FL_DISC | FL_EXACT)) continue;
      if (cur >= R) {
        S[i] = exact_sum(&I, i);
        fl[i] |= FL_EXACT;
        st->coord_evals += exact_cost(&I, T[cur - 1]);
        st->exact_points += 1;
      } else {
        S[i] += sampled_sum(&I, p->seed, i, T[cur - 1], T[cur]);
        ri[i] = (uint8_t)cur;
        st->coord_evals += T[cur] - T[cur - 1];
      }
    }
  }

  if (finished) {
    int64_t np = 0;
    for (int64_t i = 0; i < n; ++i)
      if (!(fl[i] & FL_DISC)) ++np;
    if (np > kh) {
      /* Oversized stop (only exact undecided and accepted points remain):
       * give the accepted points their exact distances too, so that the
       * k+h smallest by (d, index) contain a k-NN set even under ties. */
      for (int64_t i = 0; i < n; ++i) {
        if ((fl[i] & FL_DISC) || (fl[i] & FL_EXACT)) continue;
        S[i] = exact_sum(&I, i);
        fl[i] |= FL_EXACT;
        st->coord_evals += exact_cost(&I, T[ri[i]]);
        st->exact_points += 1;
      }
    }
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (fl[i] & FL_DISC) continue;
      int64_t Tn = (fl[i] & FL_EXACT) ? m : T[ri[i]];
      ki[c].key = dhat_of(&I, S[i], Tn);
      ki[c].idx = i;
      ++c;
    }
    qsort(ki, (size_t)c, sizeof(keyidx_t), cmp_keyidx);
    int64_t outc = c < kh ? c : kh;
    for (int64_t a = 0; a < outc; ++a) out_idx[a] = ki[a].idx;
    st->count = (int32_t)outc;
  }

  if (S_dump) memcpy(S_dump, S, (size_t)n * sizeof(int64_t));
  if (fl_dump) memcpy(fl_dump, fl, (size_t)n);
  if (ri_dump) memcpy(ri_dump, ri, (size_t)n);
  free(S); free(fl); free(ri); free(ucb); free(lcb); free(tmp); free(ki);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Naive brute force (Section 3): all distances, then sort.             */
/* ------------------------------------------------------------------ */
double orc_exact_dist(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                      const void *q, int64_t i) {
  (void)n;
  if (dtype == ORC_U8) {
    const uint8_t *xu = (const uint8_t *)X, *qu = (const uint8_t *)q;
    int64_t s = 0;
    for (int64_t j = 0; j < m; ++j) {
      int64_t d = (int64_t)xu[i * m + j] - (int64_t)qu[j];
      s += metric == ORC_L1 ? (d < 0 ? -d : d) : d * d;
    }
    return (double)s;
  }
  const float *xf = (const float *)X, *qf = (const float *)q;
  double s = 0.0;
  for (int64_t j = 0; j < m; ++j) {
    double d = (double)xf[i * m + j] - (double)qf[j];
    s += metric == ORC_L1 ? fabs(d) : d * d;
  }
  return s;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, sequential, as published (Section 4).                   */
/* The order of the points by (d^, index) is kept in an array and fixed  */
/* up after each of the (at most two) updates of an iteration: O(n) per */
/* iteration instead of the paper's heaps (Section 4.1), same decisions. */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t *S, *T;
  uint8_t *ex;
  double *dh, *al;
} alg1_state_t;

static int before(const alg1_state_t *A, int64_t a, int64_t b) {
  if (A->dh[a] != A->dh[b]) return A->dh[a] < A->dh[b];
  return a < b;
}

/* moves point i (whose d^ changed) to its place in ord[], pos[] the inverse */
static void reposition(const alg1_state_t *A, int64_t *ord, int64_t *pos, int64_t n, int64_t i) {
  int64_t p = pos[i];
  while (p > 0 && before(A, i, ord[p - 1])) {
    ord[p] = ord[p - 1];
    pos[ord[p]] = p;
    --p;
  }
  while (p + 1 < n && before(A, ord[p + 1], i)) {
    ord[p] = ord[p + 1];
    pos[ord[p]] = p;
    ++p;
  }
  ord[p] = i;
  pos[i] = p;
}

int32_t orc_alg1(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                 const void *q, int32_t k, const orc_params *p, int64_t max_iter,
                 int64_t *out_idx, orc_stats *st, int64_t *T_out) {
  if (!X || !q || !p || !out_idx || !st || n < 1 || m < 1 || k < 1) return -1;
  if (dtype != ORC_U8 && dtype != ORC_F32) return -1;
  if (!(p->delta > 0.0 && p->delta < 1.0)) return -1;
  if (p->alpha_kind < 0 || p->alpha_kind > 2) return -1;
  if (p->alpha_kind == 2 && !(p->c_alpha > 0.0)) return -1;
  const double theta = p->theta_exact == 0.0f ? 1.0 : (double)p->theta_exact;
  if (!(theta > 0.0)) return -1;
  const int64_t h = p->h < 0 ? (int64_t)k : p->h;
  const int64_t kh = (int64_t)k + h;
  memset(st, 0, sizeof(*st));
  for (int64_t a = 0; a < kh; ++a) out_idx[a] = -1;
  if (n <= kh) {
    for (int64_t i = 0; i < n; ++i) {
      out_idx[i] = i;
      if (T_out) T_out[i] = 0;
    }
    st->count = (int32_t)n;
    return 0;
  }
  inst_t I;
  memset(&I, 0, sizeof(I));
  I.n = n; I.m = m; I.dtype = dtype; I.metric = metric;
  if (dtype == ORC_U8) { I.xu = (const uint8_t *)X; I.qu = (const uint8_t *)q; }
  else { I.xf = (const float *)X; I.qf = (const float *)q; }
  int32_t F;
  int sc = orc_scaling(X, n, m, dtype, metric, q, &I.W, &F);
  if (sc < 0) return -1;
  if (sc == 1) {  /* zero range: every distance is 0 */
    for (int64_t a = 0; a < kh; ++a) out_idx[a] = a;
    st->count = (int32_t)kh;
    return 0;
  }
  I.scale = ldexp(1.0, F);
  if (p->sampling < 0 || p->sampling > 3) return -1;
  I.sampling = p->sampling;
  I.norepl = p->sampling & 1;
  double thr_d = ceil(theta * (double)m);
  const int64_t thr = thr_d >= (double)m ? m : (thr_d < 1.0 ? 1 : (int64_t)thr_d);
  alg1_state_t A;
  A.S = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  A.T = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  A.ex = (uint8_t *)calloc((size_t)n, 1);
  A.dh = (double *)calloc((size_t)n, sizeof(double));
  A.al = (double *)calloc((size_t)n, sizeof(double));
  int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  keyidx_t *tmp = (keyidx_t *)malloc(sizeof(keyidx_t) * (size_t)n);
  int64_t evals = 0, exact_pts = 0;
  /* one more sample of point i (or its exact distance at the threshold) */
  #define ALG1_SAMPLE(i) do {                                                   \
    int64_t i_ = (i);                                                           \
    A.T[i_] += 1;                                                               \
    A.S[i_] += sample_value(&I, i_, orc_coord(I.sampling, p->seed, i_, A.T[i_] - 1, m));      \
    evals += 1;                                                                 \
    if (A.T[i_] >= thr) {                                                       \
      A.S[i_] = exact_sum(&I, i_);                                              \
      A.ex[i_] = 1;                                                             \
      evals += exact_cost(&I, A.T[i_]);                                         \
      exact_pts += 1;                                                           \
      A.dh[i_] = dhat_of(&I, A.S[i_], m);                                       \
      A.al[i_] = 0.0;                                                           \
    } else {                                                                    \
      A.dh[i_] = dhat_of(&I, A.S[i_], A.T[i_]);                                 \
      A.al[i_] = orc_alpha(p->alpha_kind, A.T[i_], n, p->delta, p->c_alpha);    \
    }                                                                           \
  } while (0)
  for (int64_t i = 0; i < n; ++i) ALG1_SAMPLE(i);
  for (int64_t i = 0; i < n; ++i) { tmp[i].key = A.dh[i]; tmp[i].idx = i; }
  qsort(tmp, (size_t)n, sizeof(keyidx_t), cmp_keyidx);
  for (int64_t a = 0; a < n; ++a) { ord[a] = tmp[a].idx; pos[ord[a]] = a; }
  int32_t rc = 0;
  int64_t it = 0;
  for (;;) {
    /* eq. d_ind */
    int64_t q1 = ord[0];
    for (int64_t a = 1; a < k; ++a) {
      int64_t i = ord[a];
      double v = A.dh[i] + A.al[i], w = A.dh[q1] + A.al[q1];
      if (v > w || (v == w && i < q1)) q1 = i;
    }
    int64_t q2 = ord[kh];
    for (int64_t a = kh + 1; a < n; ++a) {
      int64_t i = ord[a];
      double v = A.dh[i] - A.al[i], w = A.dh[q2] - A.al[q2];
      if (v < w || (v == w && i < q2)) q2 = i;
    }
    /* eq. termination */
    if (A.dh[q1] + A.al[q1] <= A.dh[q2] - A.al[q2]) break;
    /* eq. blowbupdef: q2 first, then the middle positions in order */
    int64_t b2 = q2;
    for (int64_t a = k; a < kh; ++a) {
      int64_t i = ord[a];
      if (A.al[i] > A.al[b2]) b2 = i;
    }
    if (++it > max_iter) { rc = -2; break; }
    const int64_t pick[2] = {q1, b2};
    for (int c = 0; c < 2; ++c) {
      const int64_t i = pick[c];
      if (A.ex[i]) continue;  /* its distance is exact already */
      ALG1_SAMPLE(i);
      reposition(&A, ord, pos, n, i);
    }
  }
  #undef ALG1_SAMPLE
  for (int64_t a = 0; a < kh; ++a) out_idx[a] = ord[a];
  st->coord_evals = evals;
  st->rounds = it > INT32_MAX ? INT32_MAX : (int32_t)it;
  st->count = (int32_t)kh;
  st->exact_points = exact_pts;
  if (T_out) for (int64_t i = 0; i < n; ++i) T_out[i] = A.ex[i] ? m : A.T[i];
  free(A.S); free(A.T); free(A.ex); free(A.dh); free(A.al);
  free(ord); free(pos); free(tmp);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 with the bookkeeping of Section 4.1 (Figure fig:heaps):   */
/* the points are split into S_close (first k by (d^, index)), S_middle  */
/* (next h) and S_far (the rest), each with its coupled heaps -- close:  */
/* max-heaps on d^ and on d^ + alpha; middle: min- and max-heap on d^    */
/* and max-heap on alpha; far: min-heaps on d^ and on d^ - alpha.  q1,   */
/* q2 and b2 are heap tops; an updated point leaves its set's heaps and  */
/* comes back with its new bounds, then extreme elements are swapped     */
/* between neighbouring sets until the (d^, index) order across the sets */
/* holds again: O(log n) per iteration after an O(n) heapify (Floyd).    */
/* Every choice breaks ties as orc_alg1 does, so both return the same.   */
/* ------------------------------------------------------------------ */
typedef int (*above_fn)(const alg1_state_t *A, int64_t a, int64_t b);

typedef struct {
  int64_t *h;   /* heap array of point indices */
  int64_t *at;  /* at[i]: position of point i in h, -1 when absent */
  int64_t len;
  above_fn above; /* above(a, b): a belongs nearer the top than b */
} iheap_t;

static int ab_dmin(const alg1_state_t *A, int64_t a, int64_t b) { return before(A, a, b); }
static int ab_dmax(const alg1_state_t *A, int64_t a, int64_t b) { return before(A, b, a); }
static int ab_ucb(const alg1_state_t *A, int64_t a, int64_t b) {  /* largest d^ + alpha, then smaller index */
  double va = A->dh[a] + A->al[a], vb = A->dh[b] + A->al[b];
  return va > vb || (va == vb && a < b);
}
static int ab_lcb(const alg1_state_t *A, int64_t a, int64_t b) {  /* smallest d^ - alpha, then smaller index */
  double va = A->dh[a] - A->al[a], vb = A->dh[b] - A->al[b];
  return va < vb || (va == vb && a < b);
}
static int ab_alpha(const alg1_state_t *A, int64_t a, int64_t b) {  /* largest alpha, then earlier by (d^, index) */
  return A->al[a] > A->al[b] || (A->al[a] == A->al[b] && before(A, a, b));
}

static void ih_set(iheap_t *H, int64_t p, int64_t i) { H->h[p] = i; H->at[i] = p; }
static void ih_up(const alg1_state_t *A, iheap_t *H, int64_t p) {
  int64_t i = H->h[p];
  while (p > 0) {
    int64_t par = (p - 1) / 2;
    if (!H->above(A, i, H->h[par])) break;
    ih_set(H, p, H->h[par]);
    p = par;
  }
  ih_set(H, p, i);
}
static void ih_down(const alg1_state_t *A, iheap_t *H, int64_t p) {
  int64_t i = H->h[p];
  for (;;) {
    int64_t c = 2 * p + 1;
    if (c >= H->len) break;
    if (c + 1 < H->len && H->above(A, H->h[c + 1], H->h[c])) ++c;
    if (!H->above(A, H->h[c], i)) break;
    ih_set(H, p, H->h[c]);
    p = c;
  }
  ih_set(H, p, i);
}
static void ih_push(const alg1_state_t *A, iheap_t *H, int64_t i) {
  H->h[H->len] = i;
  H->at[i] = H->len;
  H->len += 1;
  ih_up(A, H, H->len - 1);
}
static void ih_remove(const alg1_state_t *A, iheap_t *H, int64_t i) {
  int64_t p = H->at[i];
  H->at[i] = -1;
  H->len -= 1;
  if (p == H->len) return;
  const int64_t x = H->h[H->len];  /* the last element fills the hole, then moves up or down */
  ih_set(H, p, x);
  ih_up(A, H, p);
  if (H->at[x] == p) ih_down(A, H, p);
}
static void ih_heapify(const alg1_state_t *A, iheap_t *H) {  /* Floyd's bottom-up construction */
  for (int64_t p = 0; p < H->len; ++p) H->at[H->h[p]] = p;
  for (int64_t p = H->len / 2 - 1; p >= 0; --p) ih_down(A, H, p);
}

enum { SET_CLOSE = 0, SET_MIDDLE = 1, SET_FAR = 2 };
typedef struct {
  iheap_t c_d, c_ucb, m_dmin, m_dmax, m_al, f_d, f_lcb;
  uint8_t *set;
} alg1_heaps_t;

static void set_insert(const alg1_state_t *A, alg1_heaps_t *H, int s, int64_t i) {
  H->set[i] = (uint8_t)s;
  if (s == SET_CLOSE) { ih_push(A, &H->c_d, i); ih_push(A, &H->c_ucb, i); }
  else if (s == SET_MIDDLE) { ih_push(A, &H->m_dmin, i); ih_push(A, &H->m_dmax, i); ih_push(A, &H->m_al, i); }
  else { ih_push(A, &H->f_d, i); ih_push(A, &H->f_lcb, i); }
}
static void set_remove(const alg1_state_t *A, alg1_heaps_t *H, int64_t i) {
  int s = H->set[i];
  if (s == SET_CLOSE) { ih_remove(A, &H->c_d, i); ih_remove(A, &H->c_ucb, i); }
  else if (s == SET_MIDDLE) { ih_remove(A, &H->m_dmin, i); ih_remove(A, &H->m_dmax, i); ih_remove(A, &H->m_al, i); }
  else { ih_remove(A, &H->f_d, i); ih_remove(A, &H->f_lcb, i); }
}
/* moves i from its set to set s */
static void set_move(const alg1_state_t *A, alg1_heaps_t *H, int64_t i, int s) {
  set_remove(A, H, i);
  set_insert(A, H, s, i);
}
/* swaps extreme elements of neighbouring sets until every close point
 * precedes every middle point and every middle point every far point */
static void restore_order(const alg1_state_t *A, alg1_heaps_t *H, int64_t h) {
  for (;;) {
    int changed = 0;
    if (h > 0) {
      int64_t a = H->c_d.h[0], b = H->m_dmin.h[0];
      if (before(A, b, a)) { set_move(A, H, a, SET_MIDDLE); set_move(A, H, b, SET_CLOSE); changed = 1; }
      a = H->m_dmax.h[0]; b = H->f_d.h[0];
      if (before(A, b, a)) { set_move(A, H, a, SET_FAR); set_move(A, H, b, SET_MIDDLE); changed = 1; }
    } else {
      int64_t a = H->c_d.h[0], b = H->f_d.h[0];
      if (before(A, b, a)) { set_move(A, H, a, SET_FAR); set_move(A, H, b, SET_CLOSE); changed = 1; }
    }
    if (!changed) return;
  }
}

static int heap_alloc(iheap_t *H, int64_t n, above_fn f) {
  H->h = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  H->at = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  H->len = 0;
  H->above = f;
  if (!H->h || !H->at) return -1;
  for (int64_t i = 0; i < n; ++i) H->at[i] = -1;
  return 0;
}
static void heap_free(iheap_t *H) { free(H->h); free(H->at); }

int32_t orc_alg1_heaps(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                       const void *q, int32_t k, const orc_params *p, int64_t max_iter,
                       int64_t *out_idx, orc_stats *st, int64_t *T_out) {
  if (!X || !q || !p || !out_idx || !st || n < 1 || m < 1 || k < 1) return -1;
  if (dtype != ORC_U8 && dtype != ORC_F32) return -1;
  if (!(p->delta > 0.0 && p->delta < 1.0)) return -1;
  if (p->alpha_kind < 0 || p->alpha_kind > 2) return -1;
  if (p->alpha_kind == 2 && !(p->c_alpha > 0.0)) return -1;
  const double theta = p->theta_exact == 0.0f ? 1.0 : (double)p->theta_exact;
  if (!(theta > 0.0)) return -1;
  const int64_t h = p->h < 0 ? (int64_t)k : p->h;
  const int64_t kh = (int64_t)k + h;
  memset(st, 0, sizeof(*st));
  for (int64_t a = 0; a < kh; ++a) out_idx[a] = -1;
  if (n <= kh) {
    for (int64_t i = 0; i < n; ++i) {
      out_idx[i] = i;
      if (T_out) T_out[i] = 0;
    }
    st->count = (int32_t)n;
    return 0;
  }
  inst_t I;
  memset(&I, 0, sizeof(I));
  I.n = n; I.m = m; I.dtype = dtype; I.metric = metric;
  if (dtype == ORC_U8) { I.xu = (const uint8_t *)X; I.qu = (const uint8_t *)q; }
  else { I.xf = (const float *)X; I.qf = (const float *)q; }
  int32_t F;
  int sc = orc_scaling(X, n, m, dtype, metric, q, &I.W, &F);
  if (sc < 0) return -1;
  if (sc == 1) {  /* zero range: every distance is 0 */
    for (int64_t a = 0; a < kh; ++a) out_idx[a] = a;
    st->count = (int32_t)kh;
    return 0;
  }
  I.scale = ldexp(1.0, F);
  if (p->sampling < 0 || p->sampling > 3) return -1;
  I.sampling = p->sampling;
  I.norepl = p->sampling & 1;
  double thr_d = ceil(theta * (double)m);
  const int64_t thr = thr_d >= (double)m ? m : (thr_d < 1.0 ? 1 : (int64_t)thr_d);
  alg1_state_t A;
  A.S = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  A.T = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  A.ex = (uint8_t *)calloc((size_t)n, 1);
  A.dh = (double *)calloc((size_t)n, sizeof(double));
  A.al = (double *)calloc((size_t)n, sizeof(double));
  keyidx_t *tmp = (keyidx_t *)malloc(sizeof(keyidx_t) * (size_t)n);
  alg1_heaps_t H;
  H.set = (uint8_t *)calloc((size_t)n, 1);
  int bad = !A.S || !A.T || !A.ex || !A.dh || !A.al || !tmp || !H.set;
  bad |= heap_alloc(&H.c_d, n, ab_dmax) | heap_alloc(&H.c_ucb, n, ab_ucb);
  bad |= heap_alloc(&H.m_dmin, n, ab_dmin) | heap_alloc(&H.m_dmax, n, ab_dmax) | heap_alloc(&H.m_al, n, ab_alpha);
  bad |= heap_alloc(&H.f_d, n, ab_dmin) | heap_alloc(&H.f_lcb, n, ab_lcb);
  int32_t rc = 0;
  int64_t evals = 0, exact_pts = 0, it = 0;
  if (bad) { rc = -1; goto done; }
  /* one more sample of point i (or its exact distance at the threshold),
   * the same update as orc_alg1 */
  #define ALG1H_SAMPLE(i) do {                                                  \
    int64_t i_ = (i);                                                           \
    A.T[i_] += 1;                                                               \
    A.S[i_] += sample_value(&I, i_, orc_coord(I.sampling, p->seed, i_, A.T[i_] - 1, m));      \
    evals += 1;                                                                 \
    if (A.T[i_] >= thr) {                                                       \
      A.S[i_] = exact_sum(&I, i_);                                              \
      A.ex[i_] = 1;                                                             \
      evals += exact_cost(&I, A.T[i_]);                                         \
      exact_pts += 1;                                                           \
      A.dh[i_] = dhat_of(&I, A.S[i_], m);                                       \
      A.al[i_] = 0.0;                                                           \
    } else {                                                                    \
      A.dh[i_] = dhat_of(&I, A.S[i_], A.T[i_]);                                 \
      A.al[i_] = orc_alpha(p->alpha_kind, A.T[i_], n, p->delta, p->c_alpha);    \
    }                                                                           \
  } while (0)
  for (int64_t i = 0; i < n; ++i) ALG1H_SAMPLE(i);
  /* the initial split by (d^, index), each set's heaps built bottom-up */
  for (int64_t i = 0; i < n; ++i) { tmp[i].key = A.dh[i]; tmp[i].idx = i; }
  qsort(tmp, (size_t)n, sizeof(keyidx_t), cmp_keyidx);
  for (int64_t a = 0; a < n; ++a) {
    const int64_t i = tmp[a].idx;
    if (a < k) {
      H.set[i] = SET_CLOSE;
      H.c_d.h[H.c_d.len++] = i; H.c_ucb.h[H.c_ucb.len++] = i;
    } else if (a < kh) {
      H.set[i] = SET_MIDDLE;
      H.m_dmin.h[H.m_dmin.len++] = i; H.m_dmax.h[H.m_dmax.len++] = i; H.m_al.h[H.m_al.len++] = i;
    } else {
      H.set[i] = SET_FAR;
      H.f_d.h[H.f_d.len++] = i; H.f_lcb.h[H.f_lcb.len++] = i;
    }
  }
  ih_heapify(&A, &H.c_d); ih_heapify(&A, &H.c_ucb);
  ih_heapify(&A, &H.m_dmin); ih_heapify(&A, &H.m_dmax); ih_heapify(&A, &H.m_al);
  ih_heapify(&A, &H.f_d); ih_heapify(&A, &H.f_lcb);
  for (;;) {
    const int64_t q1 = H.c_ucb.h[0], q2 = H.f_lcb.h[0];                /* eq. d_ind */
    if (A.dh[q1] + A.al[q1] <= A.dh[q2] - A.al[q2]) break;             /* eq. termination */
    int64_t b2 = q2;                                                   /* eq. blowbupdef */
    if (h > 0 && A.al[H.m_al.h[0]] > A.al[q2]) b2 = H.m_al.h[0];
    if (++it > max_iter) { rc = -2; break; }
    const int64_t pick[2] = {q1, b2};
    for (int c = 0; c < 2; ++c) {
      const int64_t i = pick[c];
      if (A.ex[i]) continue;  /* its distance is exact already */
      const int s = H.set[i];
      set_remove(&A, &H, i);
      ALG1H_SAMPLE(i);
      set_insert(&A, &H, s, i);
    }
    restore_order(&A, &H, h);
  }
  #undef ALG1H_SAMPLE
  {  /* the returned set: close and middle, by (d^, index) */
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i)
      if (H.set[i] != SET_FAR) { tmp[c].key = A.dh[i]; tmp[c].idx = i; ++c; }
    qsort(tmp, (size_t)c, sizeof(keyidx_t), cmp_keyidx);
    for (int64_t a = 0; a < kh; ++a) out_idx[a] = tmp[a].idx;
  }
  st->coord_evals = evals;
  st->rounds = it > INT32_MAX ? INT32_MAX : (int32_t)it;
  st->count = (int32_t)kh;
  st->exact_points = exact_pts;
  if (T_out) for (int64_t i = 0; i < n; ++i) T_out[i] = A.ex[i] ? m : A.T[i];
done:
  free(A.S); free(A.T); free(A.ex); free(A.dh); free(A.al); free(tmp); free(H.set);
  heap_free(&H.c_d); heap_free(&H.c_ucb); heap_free(&H.m_dmin); heap_free(&H.m_dmax); heap_free(&H.m_al);
  heap_free(&H.f_d); heap_free(&H.f_lcb);
  return rc;
}

int32_t orc_naive(const void *X, int64_t n, int64_t m, int32_t dtype, int32_t metric,
                  const void *q, int32_t k, int64_t *out_idx, double *out_dist) {
  if (!X || !q || !out_idx || n < 1 || m < 1 || k < 1) return -1;
  if (dtype != ORC_U8 && dtype != ORC_F32) return -1;
  if (metric != ORC_L2 && metric != ORC_L1) return -1;
  keyidx_t *ki = (keyidx_t *)malloc((size_t)n * sizeof(keyidx_t));
  if (!ki) return -2;
  for (int64_t i = 0; i < n; ++i) {
    ki[i].key = orc_exact_dist(X, n, m, dtype, metric, q, i);
    ki[i].idx = i;
  }
  qsort(ki, (size_t)n, sizeof(keyidx_t), cmp_keyidx);
  for (int64_t a = 0; a < k; ++a) {
    out_idx[a] = a < n ? ki[a].idx : -1;
    if (out_dist) out_dist[a] = a < n ? ki[a].key : INFINITY;
  }
  free(ki);
  return 0;
}
