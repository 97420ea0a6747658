// knn_api.cpp -- host runtime of libknn: the C ABI of include/knn.h, the DB
// registry, the host-side schedule and confidence widths, and the slot
// engine that drives the adaptive kernels round by round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "knn_host.h"
#include "knn_prof.h"

namespace knn {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

// ------------------------------------------------------------ widths

// Section 4 footnote: beta(u, d') = log(1/d') + 3 log log(1/d') + 1.5 log(1 + log u).
// Lemma 3 (valid for every delta): beta(u, d') = 2 log(125 log(1.12 u) / d').
// Section 5: alpha(u) = sqrt(C log(1 + (1 + log u) n / delta) / u).
// alpha(u) = sqrt(2 beta(u, delta/n) / u) for the first two.
static double width(int32_t kind, int64_t u, int64_t n, double delta, double c_alpha) {
  const double du = (double)u;
  if (kind == 2) return std::sqrt(c_alpha * std::log(1.0 + (1.0 + std::log(du)) * (double)n / delta) / du);
  const double dp = delta / (double)n;
  double beta;
  if (kind == 0 && dp < 0.05) {
    const double L = std::log(1.0 / dp);
    beta = L + 3.0 * std::log(L) + 1.5 * std::log(1.0 + std::log(du));
  } else {
    beta = 2.0 * std::log(125.0 * std::log(1.12 * du) / dp);
  }
  return std::sqrt(2.0 * beta / du);
}

bool host_schedule(const knn_params &p, int64_t n, int64_t m, Sched &out, std::string &why) {
  std::memset(&out, 0, sizeof(out));
  const int32_t b0 = p.b0 == 0 ? 64 : p.b0;
  const float g = p.growth == 0.0f ? 2.0f : p.growth;
  const float th = p.theta_exact == 0.0f ? 1.0f : p.theta_exact;
  if (b0 < 4 || b0 % 4) return why = "b0 must be a positive multiple of 4", false;
  if (!(g >= 1.0f)) return why = "growth must be >= 1", false;
  if (!(th > 0.0f)) return why = "theta_exact must be > 0", false;
  if (!(p.delta > 0.0 && p.delta < 1.0)) return why = "delta must lie in (0,1)", false;
  if (p.alpha_kind < 0 || p.alpha_kind > 2) return why = "alpha_kind must be 0, 1 or 2", false;
  if (p.alpha_kind == 2 && !(p.c_alpha > 0.0)) return why = "alpha_kind 2 needs c_alpha > 0", false;
  if (p.c_exact < 0 || p.c_exact > KNN_MAX_KH) return why = "c_exact out of range", false;
  // exact threshold ceil(theta m), clipped to [1, m]
  const double thr_d = std::ceil((double)th * (double)m);
  int64_t thr = thr_d >= (double)m ? m : (int64_t)thr_d;
  if (thr < 1) thr = 1;
  int32_t R = 0;
  for (int64_t t = b0; t < thr;) {
    if (R >= kMaxRounds) return why = "round schedule longer than KNN_MAX_ROUNDS", false;
    out.T[R] = (int32_t)t;
    out.alpha[R] = width(p.alpha_kind, t, n, p.delta, p.c_alpha);
    if (!(out.alpha[R] >= 0.0)) return why = "confidence width is not a number", false;
    ++R;
    int64_t b = (int64_t)std::ceil((double)t * ((double)g - 1.0));
    b = (b + 3) / 4 * 4;
    t += b < 4 ? 4 : b;
  }
  out.R = R;
  return true;
}

// ------------------------------------------------------------ engine

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static int env_int(const char *name, int dflt) {
  const char *v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// Performance knobs (never result-defining): the DB's autotuned values when
// it has them, else the defaults, then KNN_* environment overrides.
Knobs knobs_for(const knn_db_s *db) {
  Knobs k;
  if (db && db->tune.valid) k = db->tune;
  k.ql = env_int("KNN_QL", k.ql);
  k.ql_min = env_int("KNN_QL_MIN", k.ql_min);
  k.group = env_int("KNN_GROUP", k.group);
  k.lpp = env_int("KNN_LPP", k.lpp);
  if (k.lpp < 0 || k.lpp > 64 || (k.lpp & (k.lpp - 1)) != 0) k.lpp = 0;
  k.ch_sample = std::max(1, env_int("KNN_CH_SAMPLE", k.ch_sample));
  k.stage_min = env_int("KNN_STAGE_MIN", k.stage_min);
  k.stage_rows = env_int("KNN_STAGE_ROWS", k.stage_rows);
  k.graph = env_int("KNN_GRAPH", k.graph);
  k.sparse_div = env_int("KNN_SPARSE_DIV", k.sparse_div);
  k.seq = env_int("KNN_SEQ", k.seq);
  return k;
}

// A stream-ordered pool per device that keeps its memory mapped between
// calls: the default pool hands an engine's arena back at every
// synchronisation, and mapping it again costs about half a millisecond per
// batch.  nullptr when the pool cannot be made (the default pool is used).
static hipMemPool_t engine_pool() {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) return it->second;
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
    (void)hipGetLastError();
    pool = nullptr;
  } else {
    uint64_t keep = UINT64_MAX;
    if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipMemPoolDestroy(pool);
      pool = nullptr;
    }
  }
  pools[dev] = pool;
  return pool;
}

size_t engine_slot_bytes(int64_t n, int32_t kmax, int32_t cmax) {
  const int64_t pw = part_words(n, kmax, cmax);
  return (size_t)n * (8 + 1 + 1 + 4 * 2 + 4 * 2 + 4) + (size_t)pw * 8 + sizeof(Slot) + 12 * 256;
}

int engine_create(Engine &E, knn_db_s *db, int64_t ns, int32_t kmax, int32_t cmax, int64_t qcap, int64_t nsched,
                  hipStream_t st, bool async_alloc, bool grouped, bool query_lane, int32_t seq_tlen, int32_t seq_nb) {
  const Knobs K = knobs_for(db);
  const int64_t n = db->n;
  const int64_t pw = part_words(n, kmax, cmax);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_slots = take(sizeof(Slot) * ns);
  const size_t o_ctl = take(sizeof(Ctl));
  const size_t o_qd = take(sizeof(QDesc) * qcap);
  const size_t o_sched = take(sizeof(Sched) * nsched);
  const size_t o_S = take((size_t)ns * n * 8);
  const size_t o_fl = take((size_t)ns * n);
  const size_t o_ri = take((size_t)ns * n);
  const size_t o_act = take((size_t)ns * n * 8);
  const size_t o_xa = take((size_t)ns * n * 8);
  const size_t o_acc = take((size_t)ns * n * 4);
  const size_t o_part = take((size_t)ns * pw * 8);
  const int32_t nqp = query_lane ? (int32_t)((ns + 15) / 16 * 16) : 0;
  const size_t o_qt = take((size_t)nqp * (size_t)db->m);
  const size_t o_qdl = take((size_t)nqp * (size_t)n * 5);  // round totals [n][nqp] u32, then flags [n][nqp] u8
  // the exact round of a query-lane batch as one tiled pass over (slots x points): an int8
  // GEMM for squared l2, v_sad_u8 tiles for l1
  const bool l1 = db->metric == KNN_METRIC_L1;
  const bool q8x = query_lane && db->dtype == KNN_U8 && (l1 ? db->xpad != nullptr : db->xs8 != nullptr) &&
                   db->m <= 65536;
  const size_t o_q8 = take(q8x ? (size_t)nqp * (size_t)db->mp : 0);
  const size_t o_q8n = take(q8x ? (size_t)nqp * 4 : 0);
  // a shared coordinate sequence: its coordinates, the points and queries at
  // them, and their prefix norms at the round boundaries
  const bool seq = q8x && seq_tlen > 0;
  const bool seqf = db->dtype == KNN_F32 && seq_tlen > 0;  // fp32: float copies, no norms
  const int64_t kp = (seq || seqf) ? ((int64_t)seq_tlen + 63) / 64 * 64 : 0;
  const size_t o_js = take((seq || seqf) ? (size_t)kp * 4 : 0);
  const size_t o_xs = take(seq ? (size_t)n * kp : 0);
  const size_t o_qs = take(seq ? (size_t)nqp * kp : 0);
  const size_t o_xsn = take(seq ? (size_t)seq_nb * n * 4 : 0);
  const size_t o_qsn = take(seq ? (size_t)seq_nb * nqp * 4 : 0);
  const size_t o_sflag = take(seq ? 256 : 0);
  const size_t o_xf = take(seqf ? (size_t)n * kp * 4 : 0);
  const size_t o_qf = take(seqf ? (size_t)ns * kp * 4 : 0);
  void *base = nullptr;
  if (async_alloc) {
    hipMemPool_t pool = engine_pool();
    if (pool)
      HIP_TRY(hipMallocFromPoolAsync(&base, off, pool, st));
    else
      HIP_TRY(hipMallocAsync(&base, off, st));
  } else
    HIP_TRY(hipMalloc(&base, off));
  auto at = [&](size_t o) { return (uint8_t *)base + o; };
  E.db = db;
  E.st = st;
  E.base = base;
  E.async_alloc = async_alloc;
  E.slots = (Slot *)at(o_slots);
  E.ctl = (Ctl *)at(o_ctl);
  E.qd = (QDesc *)at(o_qd);
  E.sched = (Sched *)at(o_sched);
  E.B.S = (int64_t *)at(o_S);
  E.B.fl = at(o_fl);
  E.B.ri = at(o_ri);
  E.B.act = (int32_t *)at(o_act);
  E.B.xa = (int32_t *)at(o_xa);
  E.B.acc = (int32_t *)at(o_acc);
  E.B.part = (uint64_t *)at(o_part);
  E.B.part_stride = pw;
  E.qt = query_lane ? at(o_qt) : nullptr;
  E.qsum = query_lane ? (uint32_t *)at(o_qdl) : nullptr;
  E.q8 = q8x ? (int8_t *)at(o_q8) : nullptr;
  E.q8n = q8x ? (int32_t *)at(o_q8n) : nullptr;
  E.nqp = nqp;
  E.seq = SeqBufs{};
  if (seqf) {
    E.seq.js = (uint32_t *)at(o_js);
    E.seq.xf = (float *)at(o_xf);
    E.seq.qf = (float *)at(o_qf);
    E.seq.kp = kp;
    E.seq.tlen = seq_tlen;
    E.seq.nb = seq_nb;
  }
  if (seq) {
    E.seq.js = (uint32_t *)at(o_js);
    E.seq.xs = (int8_t *)at(o_xs);
    E.seq.qs = (int8_t *)at(o_qs);
    E.seq.xn = (int32_t *)at(o_xsn);
    E.seq.qn = (int32_t *)at(o_qsn);
    E.seq.flag = (int32_t *)at(o_sflag);
    E.seq.kp = kp;
    E.seq.tlen = seq_tlen;
    E.seq.nb = seq_nb;
  }
  E.B.cand = nullptr;
  E.B.dpm = query_lane ? E.qsum : nullptr;
  E.B.dpm_stride = nqp;
  E.G.n = n;
  E.G.m = db->m;
  E.G.dtype = db->dtype;
  E.G.nslots = (int32_t)ns;
  E.G.nslots_all = (int32_t)ns;
  E.G.packed_admit = 0;
  // points per sampling block: about 1024 blocks per step over all slots
  // (single queries on small DBs still spread over the GPU), at most the
  // knob's value, at least 16
  {
    int64_t want = (n * ns + 1023) / 1024;
    want = (want + 15) / 16 * 16;
    E.G.ch_sample = (int32_t)std::max<int64_t>(16, std::min<int64_t>(K.ch_sample, want));
  }
  E.G.ch_select = 0;
  E.G.ch_decide = 0;
  E.G.lpp = K.lpp;  // 0: chosen per round from its sample count
  E.G.prof = nullptr;
  E.G.x8 = l1 ? (const int8_t *)db->xpad : db->xs8;  // (u8 DBs; f32 DBs never read it)
  E.G.xn = db->norm_i;
  E.G.mp = db->mp;
  E.G.kmax = kmax;
  E.G.metric = db->metric;
  E.G.sparse_div = K.sparse_div;
  // grouped sampling needs the shared query tile (16 rows of mp bytes) in LDS
  // (its exact rounds use the shifted int8 copy for squared l2, and fall back to
  // per-slot sums for l1)
  E.G.grouped = (grouped && db->dtype == KNN_U8 && (db->xs8 || db->metric == KNN_METRIC_L1) &&
                 16 * db->mp + 128 <= 65536 && K.group != 0)
                    ? 1
                    : 0;
  E.ns = ns;
  E.qcap = qcap;
  E.nsched = nsched;
  HIP_TRY(hipMemsetAsync(E.slots, 0, sizeof(Slot) * ns, st));
  HIP_TRY(hipMemsetAsync(E.ctl, 0, sizeof(Ctl), st));
  return KNN_OK;
}

int engine_destroy(Engine &E) {
  if (!E.base) return KNN_OK;
  hipError_t e = E.async_alloc ? hipFreeAsync(E.base, E.st) : hipFree(E.base);
  E.base = nullptr;
  if (e != hipSuccess) return fail(KNN_EDEVICE, std::string("engine free: ") + hipGetErrorString(e));
  return KNN_OK;
}

void engine_step(Engine &E, bool any_cexact, int sample_kind, int stage_rows, const QlRound *ql) {
  launch_step(E.slots, E.qd, E.sched, E.ctl, E.db->X, E.B, E.G, any_cexact, E.st, sample_kind, stage_rows, ql, E.qt,
              E.nqp, E.qsum, E.q8, E.q8n, (E.seq.xs || E.seq.xf) ? &E.seq : nullptr);
}

int make_qdesc(const knn_db_s *db, int32_t k, const knn_params &pp, QDesc &d, Sched &sc) {
  if (k < 1) return fail(KNN_EINVAL, "k must be >= 1");
  const int64_t h = pp.h < 0 ? k : pp.h;
  const int64_t kh = k + h;
  if (kh > KNN_MAX_KH) return fail(KNN_EINVAL, "k + h exceeds KNN_MAX_KH");
  std::string why;
  if (!host_schedule(pp, db->n, db->m, sc, why)) return fail(KNN_EINVAL, why);
  std::memset(&d, 0, sizeof(d));
  d.seed = pp.seed;
  d.k = k;
  d.kh = (int32_t)kh;
  d.c_exact = pp.c_exact;
  // samples s / W lie in [0,1]: u8 (x - q)^2 <= 255^2, |x - q| <= 255; f32: k_prep_f32
  d.W = db->dtype == KNN_U8 ? (db->metric == KNN_METRIC_L1 ? 255.0 : 65025.0) : 0.0;
  d.F = 0;
  d.trivial = kh >= db->n ? 1 : 0;
  if (pp.sampling < 0 || pp.sampling > 3) return fail(KNN_EINVAL, "sampling must be 0, 1, 2 or 3");
  d.norepl = pp.sampling & 1;
  d.shared = pp.sampling >> 1;
  return KNN_OK;
}

struct Prepared {
  std::vector<QDesc> qd;
  std::vector<Sched> sched;
  int32_t kmax = 1, cmax = 0, rmax = 0;
  bool any_cexact = false;
};

static int prepare(knn_db_s *db, const void *dq, int64_t nq, const int32_t *host_k, const knn_params *p,
                   int64_t np, int64_t *out_idx, int64_t out_stride, int32_t *out_count, knn_stats *out_stats,
                   Prepared &P) {
  const int64_t n = db->n, m = db->m;
  const int elem = db->dtype == KNN_U8 ? 1 : 4;
  std::map<std::string, int> seen;
  P.qd.resize(nq);
  for (int64_t q = 0; q < nq; ++q) {
    const knn_params &pp = p[np == 1 ? 0 : q];
    QDesc &d = P.qd[q];
    Sched sc;
    int rc = make_qdesc(db, host_k[q], pp, d, sc);
    if (rc != KNN_OK) return rc;
    if (out_stride < std::min<int64_t>(d.kh, n)) return fail(KNN_EINVAL, "out_stride smaller than k + h");
    std::string key((const char *)&sc, sizeof(Sched));
    auto it = seen.find(key);
    if (it == seen.end()) {
      d.sched = (int32_t)P.sched.size();
      P.sched.push_back(sc);
      seen.emplace(key, d.sched);
      P.rmax = std::max(P.rmax, sc.R);
    } else {
      d.sched = it->second;
    }
    d.q = (const uint8_t *)dq + q * m * elem;
    d.out_idx = out_idx + q * out_stride;
    d.out_count = out_count + q;
    d.out_stats = out_stats ? out_stats + q : nullptr;
    d.out_stride = out_stride;
    P.kmax = std::max(P.kmax, d.k);
    P.cmax = std::max(P.cmax, d.c_exact);
    if (d.c_exact > 0) P.any_cexact = true;
  }
  return KNN_OK;
}

// A query-lane batch that keeps its sums point-major (see launch_lockstep)
// and whose queries share one coordinate sequence runs its rounds on copies
// of the points and queries gathered at the sequence's coordinates: the
// samples they hold (the last sampled target; with the permutation, all m,
// so the exact round adds the rest) and the norm boundaries.
static void seq_geometry(const knn_db_s *db, const Prepared &P, const Knobs &K, bool query_lane, bool same,
                         int64_t nq, int64_t ns, int32_t &tlen, int32_t &nb) {
  tlen = nb = 0;
  if (!K.seq || P.qd.empty() || !P.qd[0].shared || P.sched.size() != 1) return;
  if (db->dtype == KNN_F32) {
    // a lock-step fp32 batch whose queries share seed and draw kind: every
    // round as tiles over the float copies
    if (!same || nq > ns) return;
  } else if (!query_lane || P.any_cexact || P.kmax + 1 > kPmMaxK1) {
    return;
  }
  const int32_t R = P.sched[0].R;
  if (P.qd[0].norepl) {
    tlen = (int32_t)db->m;
    nb = R + 2;
  } else if (R > 0) {
    tlen = P.sched[0].T[R - 1];
    nb = R + 1;
  }
}

// The launches of a batch whose queries all start together: (float
// query prep,) first admission, (query-lane transposed queries,) then one
// step per round.  With one shared schedule, step t runs round t for all
// of them.  Used eagerly and under graph capture.
static void launch_lockstep(Engine &E, const Prepared &P, int64_t nq, const Knobs &K, hipStream_t st) {
  knn_db_s *db = E.db;
  const int64_t n = db->n, m = db->m;
  if (db->dtype == KNN_F32) launch_prep_f32(E.qd, (int32_t)nq, n, m, db->lo, db->hi, db->metric, st);
  launch_admit(E.slots, E.qd, E.sched, E.ctl, db->X, E.B, E.G, st, true);
  const bool lockstep = P.sched.size() == 1;
  // Query-lane batches whose every round runs the fused fold + selection (no
  // candidate-exact, k + 1 <= 128) and whose exact round is one tiled pass
  // read the sets from the flags alone: no per-slot point lists are built
  E.G.flagsets = (E.qt && E.q8 && lockstep && !P.any_cexact && P.kmax + 1 <= kPmMaxK1) ? 1 : 0;
  // one coordinate sequence for every point: the points and queries gathered
  // at its coordinates once, then every round is a range of their columns
  // (the transposed queries of the query-lane sampler are then not read)
  const bool seq = E.seq.xs && E.G.flagsets;
  if (E.qt && !seq) launch_build_qt(E.slots, (int32_t)E.ns, m, E.nqp, E.qt, st);
  if (E.q8) launch_build_q8(E.slots, (int32_t)E.ns, m, db->mp, E.q8, E.q8n, db->metric, st);
  const bool seqf = E.seq.xf != nullptr && lockstep;
  if (seqf) {
    const int tk = prof_begin(PROF_QL_AUX, st);
    launch_seq_prepare_f32(E.slots, (int32_t)E.ns, (const float *)db->X, n, m, P.qd[0].seed, P.qd[0].norepl, E.seq,
                           st);
    prof_end(tk, st, 0.0);
    prof_add_host(1, (uint64_t)E.seq.tlen);
  }
  // The points' rows are gathered in up to three parts: the columns of the
  // first rounds [0, seq_ca) up front (rounds with T <= max(2048, 2 T_0));
  // the later sampled rounds' columns
  // [seq_ca, seq_c1) before round seq_ra + 1, if a slot is still running;
  // the exact round's [seq_c1, kp) before it, if a slot is still dense.
  // (A batch whose slots finish early never reads the later columns; each
  // part reads the point rows once more.)  Their norms follow each part.
  int64_t seq_ca = 0, seq_c1 = 0;
  int32_t seq_ra = -1, seq_ba = 1;
  const int seq_R = P.sched[0].R;
  if (seq && seq_R > 0) {
    const int64_t tcap = std::max<int64_t>(2048, 2 * (int64_t)P.sched[0].T[0]);
    seq_ra = 0;
    while (seq_ra + 1 < seq_R && (int64_t)P.sched[0].T[seq_ra + 1] <= tcap) ++seq_ra;
    seq_ca = std::min<int64_t>(E.seq.kp, ((int64_t)P.sched[0].T[seq_ra] + 63) / 64 * 64);
    seq_c1 = std::min<int64_t>(E.seq.kp, ((int64_t)P.sched[0].T[seq_R - 1] + 63) / 64 * 64);
    seq_ba = seq_ra + 2;  // boundaries b <= seq_ra + 1 lie below seq_ca
    // deferring the exact round's columns costs one more read of the point
    // rows when they are needed: only worth it when they are half of m or more
    if (2 * (E.seq.kp - seq_c1) < m) {
      if (seq_ca == seq_c1) seq_ca = E.seq.kp;
      seq_c1 = E.seq.kp;
    }
  }
  if (seq) {
    const int tk = prof_begin(PROF_QL_AUX, st);
    launch_seq_prepare(E.slots, E.sched, (int32_t)E.ns, E.nqp, db->X, n, m, P.qd[0].seed, P.qd[0].norepl,
                       db->metric, E.seq, db->norm_i, E.q8n, seq_ca, seq_ba, st);
    prof_end(tk, st, 0.0);
    prof_add_host(1, (uint64_t)E.seq.tlen);  // its distinct draws: one sequence for the whole batch
  }
  // long rounds of grouped sampling read whole point rows into LDS
  const int stage_rows = E.G.grouped ? stage_rows_for(m, db->mp, K.stage_rows) : 0;
  for (int t = 0; t < P.rmax + 1; ++t) {
    int stage = 0;
    if (lockstep && stage_rows > 0 && t < P.sched[0].R) {
      const int64_t b_r = P.sched[0].T[t] - (t ? P.sched[0].T[t - 1] : 0);
      if (b_r >= K.stage_min) stage = stage_rows;
    }
    QlRound qr{};
    // the round's descriptor: query-lane batches, and lock-step fp32 batches
    // (whose rounds run as tiles)
    const bool ql = (E.qt && (t < P.sched[0].R || (t == P.sched[0].R && E.q8))) || seqf;
    if (ql) {
      qr.seed = P.qd[0].seed;
      qr.norepl = P.qd[0].norepl;
      qr.shared = P.qd[0].shared;
      qr.exact = t >= P.sched[0].R;
      qr.t0 = (t && !qr.exact) ? (uint32_t)P.sched[0].T[t - 1] : 0u;
      qr.t1 = qr.exact ? 0u : (uint32_t)P.sched[0].T[t];
      if ((seq || seqf) && qr.exact && qr.norepl) {  // the coordinates not sampled yet
        qr.t0 = t ? (uint32_t)P.sched[0].T[t - 1] : 0u;
        qr.t1 = (uint32_t)m;
      }
      qr.cur = t;
      qr.impl = t == 0;
    }
    if (seq && ql && !qr.exact && t == seq_ra + 1) {
      const int tk = prof_begin(PROF_QL_AUX, st);
      launch_seq_gather_more(E.slots, (int32_t)E.ns, E.sched, db->X, n, m, db->metric, E.seq, seq_ca, seq_c1, seq_ba,
                             seq_R + 1, 0, db->norm_i, st);
      prof_end(tk, st, 0.0);
    }
    if (seq && ql && qr.exact && qr.norepl) {
      const int tk = prof_begin(PROF_QL_AUX, st);
      launch_seq_gather_more(E.slots, (int32_t)E.ns, E.sched, db->X, n, m, db->metric, E.seq, seq_c1, E.seq.kp,
                             std::max(seq_ba, seq_R + 1), seq_R + 2, 1, db->norm_i, st);
      prof_end(tk, st, 0.0);
    }
    engine_step(E, P.any_cexact, (lockstep && t == P.rmax) ? 1 : 0, stage, ql ? &qr : nullptr);
  }
}

// Resets the slots and the control block of a cached engine at the start of
// a graph replay (a kernel, not a memset node).
__global__ void k_reset_engine(uint32_t *slots_words, int64_t nwords, Ctl *ctl, const Ctl *ctl_init) {
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += (int64_t)gridDim.x * blockDim.x)
    slots_words[w] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *ctl = *ctl_init;
}

// A cached engine for repeated batches of one shape, with its launch
// sequence captured once in a hipGraph and replayed per call.
struct Plan {
  std::string key;
  Engine E;
  Ctl *ctl_init = nullptr;     // device copy of the control block at the start of a batch
  QDesc *qd_host = nullptr;    // pinned staging of the per-call query table
  hipEvent_t staged = nullptr; // the previous call's upload has left qd_host
  hipEvent_t done = nullptr;   // the previous replay has finished with the engine
  hipStream_t cap = nullptr;   // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (E.base) (void)hipDeviceSynchronize();
    engine_destroy(E);
    if (ctl_init) (void)hipFree(ctl_init);
    if (qd_host) (void)hipHostFree(qd_host);
    if (staged) (void)hipEventDestroy(staged);
    if (done) (void)hipEventDestroy(done);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

void plan_free(Plan *p) { delete p; }

static int run_graph(knn_db_s *db, const Prepared &P, int64_t nq, int64_t ns, bool same, bool query_lane,
                     const Knobs &K, hipStream_t st) {
  std::string key;
  auto put = [&](const void *v, size_t b) { key.append((const char *)v, b); };
  const int32_t hdr[8] = {(int32_t)nq, (int32_t)ns, P.kmax, P.cmax, P.rmax, (int32_t)P.any_cexact, (int32_t)same,
                          (int32_t)query_lane};
  put(hdr, sizeof(hdr));
  put(&K, sizeof(K));
  put(P.sched.data(), sizeof(Sched) * P.sched.size());
  if (query_lane || (same && P.qd[0].shared)) {  // the shared seed and draw kind are arguments of captured launches
    const uint64_t sd[2] = {P.qd[0].seed, (uint64_t)P.qd[0].norepl | ((uint64_t)P.qd[0].shared << 1)};
    put(sd, sizeof(sd));
  }
  Plan *pl = db->plan;
  if (!pl || pl->key != key) {
    if (pl) {
      plan_free(pl);
      db->plan = nullptr;
    }
    std::unique_ptr<Plan> np(new Plan());
    np->key = key;
    int32_t seq_tlen = 0, seq_nb = 0;
    seq_geometry(db, P, K, query_lane, same, nq, ns, seq_tlen, seq_nb);
    int rc = engine_create(np->E, db, ns, P.kmax, P.cmax, nq, (int64_t)P.sched.size(), st, false, same, query_lane,
                           seq_tlen, seq_nb);
    if (rc != KNN_OK) return rc;
    Ctl ctl;
    std::memset(&ctl, 0, sizeof(ctl));
    ctl.nq = (int32_t)nq;
    ctl.qcap = (int32_t)nq;
    ctl.next_query = (int32_t)std::min<int64_t>(ns, nq);  // the first admission hands query s to slot s
    HIP_TRY(hipMalloc(&np->ctl_init, sizeof(Ctl)));
    HIP_TRY(hipHostMalloc(&np->qd_host, sizeof(QDesc) * nq));
    HIP_TRY(hipEventCreateWithFlags(&np->staged, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&np->done, hipEventDisableTiming));
    HIP_TRY(hipStreamCreateWithFlags(&np->cap, hipStreamNonBlocking));
    HIP_TRY(hipMemcpyAsync(np->ctl_init, &ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(np->E.sched, P.sched.data(), sizeof(Sched) * P.sched.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    Engine &E = np->E;
    E.st = np->cap;
    HIP_TRY(hipStreamBeginCapture(np->cap, hipStreamCaptureModeThreadLocal));
    const int64_t nwords = (int64_t)sizeof(Slot) * ns / 4;
    hipLaunchKernelGGL(k_reset_engine, dim3((unsigned)std::min<int64_t>((nwords + 255) / 256, 1024)), dim3(256), 0,
                       np->cap, reinterpret_cast<uint32_t *>(E.slots), nwords, E.ctl, np->ctl_init);
    launch_lockstep(E, P, nq, K, np->cap);
    hipError_t e = hipStreamEndCapture(np->cap, &np->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&np->exec, np->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(KNN_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    pl = np.release();
    db->plan = pl;
  }
  HIP_TRY(hipEventSynchronize(pl->staged));  // the staging buffer is free again
  std::memcpy(pl->qd_host, P.qd.data(), sizeof(QDesc) * nq);
  HIP_TRY(hipStreamWaitEvent(st, pl->done, 0));  // a replay on another stream must finish first
  HIP_TRY(hipMemcpyAsync(pl->E.qd, pl->qd_host, sizeof(QDesc) * nq, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(pl->staged, st));
  HIP_TRY(hipGraphLaunch(pl->exec, st));
  HIP_TRY(hipEventRecord(pl->done, st));
  return KNN_OK;
}

// Runs the slot engine over the prepared queries.  stop_after > 0 (debug
// state dump) runs every query in a slot of its own, freezes each after
// that many decide steps and leaves the engine allocated in *keep.
static int run_engine(knn_db_s *db, Prepared &P, int64_t nq, hipStream_t st, int32_t stop_after, Engine *keep,
                      bool allow_graph = true) {
  const int64_t n = db->n, m = db->m;
  const Knobs K = knobs_for(db);
  const size_t per_slot = engine_slot_bytes(n, P.kmax, P.cmax);
  size_t freeb = 0, totb = 0;
  HIP_TRY(hipMemGetInfo(&freeb, &totb));
  size_t budget = (size_t)(freeb * 0.5);
  const size_t cap = (size_t)env_int("KNN_SLOT_BUDGET_MB", 65536) << 20;
  budget = std::min(budget, cap);
  int64_t ns = (int64_t)(budget / per_slot);
  ns = std::min<int64_t>(ns, nq);
  ns = std::min<int64_t>(ns, env_int("KNN_MAX_SLOTS", 65535));
  if (ns < 1) return fail(KNN_ENOMEM, "not enough device memory for one query slot");
  if (stop_after > 0 && ns < nq) return fail(KNN_ENOMEM, "the queries of a state dump do not fit at once");
  // queries that share seed and schedule draw identical coordinates: let
  // the sampling kernel serve them in groups
  bool same = true;
  for (int64_t q = 1; q < nq && same; ++q)
    same = P.qd[q].seed == P.qd[0].seed && P.qd[q].sched == P.qd[0].sched && P.qd[q].norepl == P.qd[0].norepl &&
           P.qd[q].shared == P.qd[0].shared;
  // More queries than slots, all with one seed and schedule: consecutive
  // lock-step batches of at most ns queries (equal sizes but the last, which
  // runs uncaptured so that the cached graph keeps the common shape), each on
  // the lock-step paths, instead of recycling slots round by round.
  if (same && nq > ns && P.sched.size() == 1 && stop_after == 0 && !keep) {
    const int64_t nch = (nq + ns - 1) / ns, c = (nq + nch - 1) / nch;
    for (int64_t q0 = 0; q0 < nq; q0 += c) {
      const int64_t len = std::min(c, nq - q0);
      Prepared Pc;
      Pc.qd.assign(P.qd.begin() + q0, P.qd.begin() + q0 + len);
      Pc.sched = P.sched;
      Pc.kmax = P.kmax;
      Pc.cmax = P.cmax;
      Pc.rmax = P.rmax;
      Pc.any_cexact = P.any_cexact;
      const int rc = run_engine(db, Pc, len, st, 0, nullptr, allow_graph && len == c);
      if (rc != KNN_OK) return rc;
    }
    return KNN_OK;
  }
  // Query-lane sampling: with every query in flight at once (nq <= ns) and
  // one seed and schedule, all slots run the same round at each step, so a
  // wave can serve one point for many slots at a time.
  const bool query_lane = same && db->dtype == KNN_U8 && m < 65536 && (nq <= ns || stop_after > 0) &&
                          P.sched.size() == 1 && ns >= K.ql_min && K.ql != 0;
  // Repeated batches of one shape replay a captured launch sequence on a
  // cached engine (not with timing on, and not for LDS-staged rounds).
  if (allow_graph && K.graph != 0 && stop_after == 0 && !keep && nq <= ns && P.sched.size() == 1 && !prof_enabled() &&
      K.stage_min >= (1 << 30))
    return run_graph(db, P, nq, ns, same, query_lane, K, st);
  Engine E;
  int32_t seq_tlen = 0, seq_nb = 0;
  seq_geometry(db, P, K, query_lane, same, nq, ns, seq_tlen, seq_nb);
  int rc = engine_create(E, db, ns, P.kmax, P.cmax, nq, (int64_t)P.sched.size(), st, true, same, query_lane, seq_tlen,
                         seq_nb);
  if (rc != KNN_OK) return rc;
  Ctl ctl;
  std::memset(&ctl, 0, sizeof(ctl));
  ctl.nq = (int32_t)nq;
  ctl.qcap = (int32_t)nq;
  ctl.stop_after = stop_after;
  ctl.next_query = (int32_t)std::min<int64_t>(ns, nq);  // the first admission hands query s to slot s
  auto chk = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && rc == KNN_OK)
      rc = fail(e == hipErrorOutOfMemory ? KNN_ENOMEM : KNN_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  {  // the control block, query descriptors and schedules through the DB's pinned staging buffer
    std::lock_guard<std::mutex> lk(db->stage_mu);
    const size_t b_ctl = align_up(sizeof(Ctl), 256), b_qd = align_up(sizeof(QDesc) * nq, 256);
    const size_t b_sc = sizeof(Sched) * P.sched.size(), need = b_ctl + b_qd + b_sc;
    if (db->stage_done)
      chk(hipEventSynchronize(db->stage_done), "staging wait");  // the previous batch's copies are done
    else
      chk(hipEventCreateWithFlags(&db->stage_done, hipEventDisableTiming), "staging event");
    if (rc == KNN_OK && need > db->stage_cap) {
      if (db->stage) (void)hipHostFree(db->stage);
      db->stage = nullptr;
      db->stage_cap = 0;
      chk(hipHostMalloc(&db->stage, need), "staging buffer");
      if (rc == KNN_OK) db->stage_cap = need;
    }
    if (rc == KNN_OK) {
      uint8_t *h = static_cast<uint8_t *>(db->stage);
      std::memcpy(h, &ctl, sizeof(Ctl));
      std::memcpy(h + b_ctl, P.qd.data(), sizeof(QDesc) * nq);
      std::memcpy(h + b_ctl + b_qd, P.sched.data(), b_sc);
      chk(hipMemcpyAsync(E.ctl, h, sizeof(Ctl), hipMemcpyHostToDevice, st), "copy ctl");
      chk(hipMemcpyAsync(E.qd, h + b_ctl, sizeof(QDesc) * nq, hipMemcpyHostToDevice, st), "copy queries");
      chk(hipMemcpyAsync(E.sched, h + b_ctl + b_qd, b_sc, hipMemcpyHostToDevice, st), "copy schedules");
      chk(hipEventRecord(db->stage_done, st), "staging record");
    }
  }
  const bool lockstep = nq <= ns || stop_after > 0;
  if (rc == KNN_OK) {
    if (lockstep) {
      launch_lockstep(E, P, nq, K, st);
      chk(hipGetLastError(), "launch");
    } else {
      if (db->dtype == KNN_F32) launch_prep_f32(E.qd, (int32_t)nq, n, m, db->lo, db->hi, db->metric, st);
      launch_admit(E.slots, E.qd, E.sched, E.ctl, db->X, E.B, E.G, st, true);
      chk(hipGetLastError(), "launch");
      // slots are recycled on the device; poll until every query is done
      const int steps_gen = P.rmax + 1;
      const int64_t max_gen = ((nq + ns - 1) / ns + 1) * (P.rmax + 2);
      int64_t gen = 0;
      for (;;) {
        for (int t = 0; t < steps_gen; ++t) engine_step(E, P.any_cexact);
        chk(hipGetLastError(), "launch");
        int32_t done = 0;
        chk(hipMemcpyAsync(&done, &E.ctl->done, sizeof(int32_t), hipMemcpyDeviceToHost, st), "poll");
        chk(hipStreamSynchronize(st), "poll sync");
        if (rc != KNN_OK || done >= nq) break;
        if (++gen > max_gen) {
          rc = fail(KNN_EDEVICE, "adaptive engine made no progress");
          break;
        }
      }
    }
  }
  if (keep && rc == KNN_OK) {
    *keep = E;
    return KNN_OK;  // caller frees
  }
  const int rc2 = engine_destroy(E);  // (a stream-ordered free)
  // a batch with every query in flight at once is stream-ordered: its host
  // data went through the staging buffer, so the call returns without
  // waiting; the polled form has synchronised already
  if (!lockstep || rc != KNN_OK) chk(hipStreamSynchronize(st), "hipStreamSynchronize");
  return rc != KNN_OK ? rc : rc2;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace knn

using namespace knn;

extern "C" {

void knn_params_default(knn_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->h = -1;
  p->delta = 0.01;
  p->seed = 0;
  p->alpha_kind = 0;
  p->c_alpha = 0.0;
  p->b0 = 64;
  p->growth = 2.0f;
  p->theta_exact = 1.0f;
  p->c_exact = 0;
  p->sampling = 0;
}

const char *knn_last_error(void) { return g_err.c_str(); }

const char *knn_version(void) { return "libknn 0.1 (gfx950)"; }

int knn_db_create(const void *dev_points, int64_t n, int64_t m, knn_dtype dt, int32_t flags, knn_db *out) {
  if (!out || !dev_points) return fail(KNN_EINVAL, "NULL argument");
  if (n < 1 || m < 1 || n >= (int64_t)1 << 31 || m >= (int64_t)1 << 31)
    return fail(KNN_EINVAL, "n and m must lie in [1, 2^31)");
  if (dt != KNN_U8 && dt != KNN_F32) return fail(KNN_EINVAL, "bad dtype");
  if (flags & ~(KNN_DB_COPY | KNN_DB_L1)) return fail(KNN_EINVAL, "bad flags");
  knn_db_s *db = new knn_db_s();
  db->n = n;
  db->m = m;
  db->dtype = dt;
  db->metric = (flags & KNN_DB_L1) ? KNN_METRIC_L1 : KNN_METRIC_L2;
  const size_t bytes = (size_t)n * m * (dt == KNN_U8 ? 1 : 4);
  hipStream_t st = nullptr;
  int rc = KNN_OK;
  if ((flags & KNN_DB_COPY) || !aligned16(dev_points)) {
    hipError_t e = hipMalloc(&db->owned, bytes);
    if (e == hipSuccess) e = hipMemcpy(db->owned, dev_points, bytes, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
      rc = fail(e == hipErrorOutOfMemory ? KNN_ENOMEM : KNN_EDEVICE, std::string("copy DB: ") + hipGetErrorString(e));
    }
    db->X = (const uint8_t *)db->owned;
  } else {
    db->X = (const uint8_t *)dev_points;
  }
  if (rc == KNN_OK && dt == KNN_F32) rc = db_range_f32((const float *)db->X, n * m, &db->lo, &db->hi, st);
  if (rc == KNN_OK) rc = naive_prepare_db(db, st);
  if (rc != KNN_OK) {
    naive_free_db(db);
    if (db->owned) (void)hipFree(db->owned);
    delete db;
    return rc;
  }
  *out = db;
  return KNN_OK;
}

int knn_db_destroy(knn_db db) {
  if (!db) return fail(KNN_EINVAL, "NULL db");
  if (db->users.load() > 0) return fail(KNN_EBUSY, "DB is held by a session");
  (void)hipDeviceSynchronize();
  if (db->plan) plan_free(db->plan);
  if (db->stage) (void)hipHostFree(db->stage);
  if (db->stage_done) (void)hipEventDestroy(db->stage_done);
  naive_free_db(db);
  if (db->owned) (void)hipFree(db->owned);
  delete db;
  return KNN_OK;
}

int knn_db_info(knn_db db, int64_t *n, int64_t *m, int32_t *dtype) {
  if (!db) return fail(KNN_EINVAL, "NULL db");
  if (n) *n = db->n;
  if (m) *m = db->m;
  if (dtype) *dtype = db->dtype;
  return KNN_OK;
}

int knn_db_metric(knn_db db, int32_t *metric) {
  if (!db || !metric) return fail(KNN_EINVAL, "NULL argument");
  *metric = db->metric;
  return KNN_OK;
}

int knn_schedule(const knn_params *p, int64_t n, int64_t m, int32_t *host_T, double *host_alpha, int32_t *R) {
  if (!p || !host_T || !host_alpha || !R) return fail(KNN_EINVAL, "NULL argument");
  if (n < 1 || m < 1) return fail(KNN_EINVAL, "n and m must be >= 1");
  Sched sc;
  std::string why;
  if (!host_schedule(*p, n, m, sc, why)) return fail(KNN_EINVAL, why);
  for (int r = 0; r < kMaxRounds; ++r) {
    host_T[r] = sc.T[r];
    host_alpha[r] = sc.alpha[r];
  }
  *R = sc.R;
  return KNN_OK;
}

int knn_adaptive(knn_db db, const void *dev_queries, int64_t nq, const int32_t *host_k, const knn_params *p,
                 int64_t np, int64_t *dev_out_idx, int64_t out_stride, int32_t *dev_out_count,
                 knn_stats *dev_out_stats, void *stream) {
  if (!db || !host_k || !p || !dev_out_idx || !dev_out_count) return fail(KNN_EINVAL, "NULL argument");
  if (nq < 0 || nq >= (int64_t)1 << 31) return fail(KNN_EINVAL, "bad nq");
  if (nq == 0) return KNN_OK;
  if (!dev_queries) return fail(KNN_EINVAL, "NULL queries");
  if (np != 1 && np != nq) return fail(KNN_EINVAL, "np must be 1 or nq");
  Prepared P;
  int rc = prepare(db, dev_queries, nq, host_k, p, np, dev_out_idx, out_stride, dev_out_count, dev_out_stats, P);
  if (rc != KNN_OK) return rc;
  std::lock_guard<std::mutex> lk(db->mu);
  return run_engine(db, P, nq, (hipStream_t)stream, 0, nullptr);
}

int knn_autotune(knn_db db, const void *dev_queries, int64_t nq, int32_t k, const knn_params *p, int32_t reps,
                 int32_t schedule_report, char *report, size_t report_len, void *stream) {
  if (!db || !dev_queries || !p || nq < 1 || k < 1) return fail(KNN_EINVAL, "bad autotune arguments");
  if (reps < 1) reps = 1;
  hipStream_t st = (hipStream_t)stream;
  const int64_t kh = k + (p->h < 0 ? k : p->h);
  const int64_t stride = std::max<int64_t>(1, std::min<int64_t>(kh, db->n));
  int64_t *d_idx = nullptr;
  int32_t *d_cnt = nullptr;
  knn_stats *d_st = nullptr;
  HIP_TRY(hipMalloc(&d_idx, sizeof(int64_t) * stride * nq));
  HIP_TRY(hipMalloc(&d_cnt, sizeof(int32_t) * nq));
  HIP_TRY(hipMalloc(&d_st, sizeof(knn_stats) * nq));
  std::vector<int32_t> ks(nq, k);
  std::vector<int64_t> ref_idx, got_idx(stride * nq);
  std::vector<int32_t> ref_cnt, got_cnt(nq);
  std::vector<knn_stats> ref_st, got_st(nq);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::string rep;
  int rc = KNN_OK;
  // one candidate: warm-up, check the output, then the mean of reps timed runs
  auto measure = [&](const knn_params &pp, double *ms, bool check) -> int {
    int r = knn_adaptive(db, dev_queries, nq, ks.data(), &pp, 1, d_idx, stride, d_cnt, d_st, st);
    if (r != KNN_OK) return r;
    HIP_TRY(hipMemcpyAsync(got_idx.data(), d_idx, sizeof(int64_t) * stride * nq, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(got_cnt.data(), d_cnt, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(got_st.data(), d_st, sizeof(knn_stats) * nq, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (check) {
      if (ref_idx.empty()) {
        ref_idx = got_idx;
        ref_cnt = got_cnt;
        ref_st = got_st;
      } else if (ref_idx != got_idx || ref_cnt != got_cnt ||
                 std::memcmp(ref_st.data(), got_st.data(), sizeof(knn_stats) * nq) != 0) {
        return fail(KNN_EDEVICE, "autotune: a performance knob changed the result");
      }
    }
    HIP_TRY(hipEventRecord(e0, st));
    for (int i = 0; i < reps; ++i) {
      r = knn_adaptive(db, dev_queries, nq, ks.data(), &pp, 1, d_idx, stride, d_cnt, d_st, st);
      if (r != KNN_OK) return r;
    }
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    return KNN_OK;
  };
  struct Cand {
    const char *name;
    Knobs k;
  };
  std::vector<Cand> cands;
  Knobs base;
  base.valid = 1;
  cands.push_back({"default", base});
  {
    Knobs c = base;
    c.ql = 0;
    cands.push_back({"grouped", c});
    c.group = 0;
    cands.push_back({"per-query", c});
    c = base;
    c.ql = 0;
    c.ch_sample = 1024;
    cands.push_back({"grouped ch1024", c});
    c.ch_sample = 4096;
    cands.push_back({"grouped ch4096", c});
    c = base;
    c.ql = 0;
    c.lpp = 16;
    cands.push_back({"grouped lpp16", c});
    c = base;
    c.graph = 0;
    cands.push_back({"default no-graph", c});
  }
  const Knobs saved = db->tune;
  double best_ms = 1e300;
  Knobs best = base;
  char line[160];
  for (const Cand &c : cands) {
    db->tune = c.k;
    double ms = 0.0;
    rc = measure(*p, &ms, true);
    if (rc != KNN_OK) break;
    std::snprintf(line, sizeof(line), "%s %.4f\n", c.name, ms);
    rep += line;
    if (ms < best_ms) {
      best_ms = ms;
      best = c.k;
    }
  }
  db->tune = rc == KNN_OK ? best : saved;
  if (rc == KNN_OK && schedule_report) {
    const int b0s[3] = {16, 64, 256};
    const float gs[2] = {1.5f, 2.0f};
    for (int b : b0s)
      for (float g : gs) {
        knn_params pp = *p;
        pp.b0 = b;
        pp.growth = g;
        double ms = 0.0;
        rc = measure(pp, &ms, false);
        if (rc != KNN_OK) break;
        std::snprintf(line, sizeof(line), "schedule b0=%d g=%.1f %.4f\n", b, (double)g, ms);
        rep += line;
      }
  }
  if (report && report_len) {
    const size_t c = std::min(report_len - 1, rep.size());
    std::memcpy(report, rep.data(), c);
    report[c] = 0;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_idx);
  (void)hipFree(d_cnt);
  (void)hipFree(d_st);
  return rc;
}

int knn_adaptive_state(knn_db db, const void *dev_queries, int64_t nq, const int32_t *host_k, const knn_params *p,
                       int64_t np, int64_t query, int32_t stop_after, int64_t *host_S, uint8_t *host_fl,
                       uint8_t *host_ri, void *stream) {
  if (!db || !dev_queries || !host_k || !p || !host_S || !host_fl || !host_ri) return fail(KNN_EINVAL, "NULL argument");
  if (nq < 1 || nq >= (int64_t)1 << 31) return fail(KNN_EINVAL, "bad nq");
  if (np != 1 && np != nq) return fail(KNN_EINVAL, "np must be 1 or nq");
  if (query < 0 || query >= nq) return fail(KNN_EINVAL, "query outside [0, nq)");
  if (stop_after < 1) return fail(KNN_EINVAL, "stop_after must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  int64_t stride = 1;
  for (int64_t q = 0; q < nq; ++q) {
    const knn_params &pp = p[np == 1 ? 0 : q];
    stride = std::max<int64_t>(stride, (int64_t)host_k[q] + (pp.h < 0 ? host_k[q] : pp.h));
  }
  stride = std::min<int64_t>(stride, std::max<int64_t>(db->n, 1));
  int64_t *d_idx = nullptr;
  int32_t *d_cnt = nullptr;
  HIP_TRY(hipMalloc(&d_idx, sizeof(int64_t) * stride * nq));
  HIP_TRY(hipMalloc(&d_cnt, sizeof(int32_t) * nq));
  Prepared P;
  int rc = prepare(db, dev_queries, nq, host_k, p, np, d_idx, stride, d_cnt, nullptr, P);
  if (rc == KNN_OK && P.qd[query].trivial) rc = fail(KNN_EINVAL, "trivial query (k + h >= n) has no state");
  Engine E;
  if (rc == KNN_OK) {
    std::lock_guard<std::mutex> lk(db->mu);
    rc = run_engine(db, P, nq, st, stop_after, &E);
    if (rc == KNN_OK) {
      // the first admission hands query q to slot q
      const int64_t n = db->n, off = query * n;
      hipError_t e = hipMemcpyAsync(host_S, E.B.S + off, n * 8, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(host_fl, E.B.fl + off, n, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(host_ri, E.B.ri + off, n, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      const int rc2 = engine_destroy(E);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) rc = fail(KNN_EDEVICE, std::string("state copy: ") + hipGetErrorString(e));
      else if (rc2 != KNN_OK) rc = rc2;
    }
  }
  (void)hipFree(d_idx);
  (void)hipFree(d_cnt);
  return rc;
}

int knn_naive(knn_db db, const void *dev_queries, int64_t nq, int32_t k, int64_t *dev_out_idx,
              double *dev_out_dist, void *stream) {
  if (!db || !dev_out_idx) return fail(KNN_EINVAL, "NULL argument");
  if (nq < 0 || nq >= (int64_t)1 << 31) return fail(KNN_EINVAL, "bad nq");
  if (k < 1 || k > KNN_MAX_KH || k > db->n) return fail(KNN_EINVAL, "k must lie in [1, min(n, KNN_MAX_KH)]");
  if (nq == 0) return KNN_OK;
  if (!dev_queries) return fail(KNN_EINVAL, "NULL queries");
  return naive_run(db, dev_queries, nq, k, dev_out_idx, dev_out_dist, (hipStream_t)stream);
}

int knn_naive_noalloc(knn_db db, const void *dev_queries, int64_t nq, int32_t k, int64_t *dev_out_idx,
                      double *dev_out_dist, void *stream) {
  if (!db || !dev_out_idx) return fail(KNN_EINVAL, "NULL argument");
  if (nq < 0 || nq >= (int64_t)1 << 31) return fail(KNN_EINVAL, "bad nq");
  if (k < 1 || k > KNN_MAX_KH || k > db->n) return fail(KNN_EINVAL, "k must lie in [1, min(n, KNN_MAX_KH)]");
  if (nq == 0) return KNN_OK;
  if (!dev_queries) return fail(KNN_EINVAL, "NULL queries");
  return naive_run_noalloc(db, dev_queries, nq, k, dev_out_idx, dev_out_dist, (hipStream_t)stream);
}

}  // extern "C"
