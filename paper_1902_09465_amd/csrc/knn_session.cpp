// knn_session.cpp -- serving session: resident DBs, memory-admitted query
// slots, and continuous batching.
//
// Each DB added to a session gets a slot engine (device state for a fixed
// number of in-flight queries, sized from the session's HBM budget) on its
// own HIP stream, device rings for query vectors, descriptors and results,
// and its own worker thread, so that DBs progress independently.  A worker
// loops:
//   1. moves submitted requests into free ring entries (uploads the queries,
//      descriptors and schedules of the whole batch, then raises the
//      engine's query count);
//   2. launches one round ("step") on the engine -- queries admitted on the
//      device join at this round boundary while the others continue where
//      they are;
//   3. synchronises its stream and collects finished queries.
// Requests therefore overlap on the device and are admitted as slots and
// memory free up; each result depends only on (query, DB, k, params).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "knn_host.h"

namespace knn {

constexpr int64_t kSessionMaxKH = 512;   // k + h limit per session request
constexpr int64_t kSessionMaxSlots = 1024;

struct Request {
  uint64_t ticket = 0;
  int32_t db_id = 0;
  std::vector<uint8_t> q;
  QDesc d{};
  QDesc dd{};           // the descriptor as uploaded (device pointers filled in)
  Sched sc{};
  bool done = false;
  int err = KNN_OK;
  std::vector<int64_t> idx;
  int32_t count = 0;
  knn_stats st{};
};

struct DbEngine {
  knn_db_s *db = nullptr;
  hipStream_t st = nullptr;
  Engine E;
  int64_t qcap = 0;
  uint8_t *dq = nullptr;       // [qcap][m * elem] query ring
  int64_t *didx = nullptr;     // [qcap][kSessionMaxKH]
  int32_t *dcnt = nullptr;     // [qcap] (-1 while running)
  knn_stats *dstats = nullptr; // [qcap]
  int32_t submitted = 0;       // queries handed to the device so far
  std::vector<Request *> ring; // request in each ring entry
  int64_t inflight = 0;
  std::deque<Request *> pending;
  std::vector<int32_t> hcnt;
  int32_t nq_host = 0;         // source of the query-count upload
  std::condition_variable cv;  // new requests for this DB
  std::thread worker;
};

}  // namespace knn

struct knn_session_s {
  size_t budget = 0, reserved = 0;
  std::mutex mu;
  std::vector<std::unique_ptr<knn::DbEngine>> dbs;
  std::unordered_map<uint64_t, knn::Request *> reqs;
  uint64_t next_ticket = 1;
  std::atomic<bool> stop{false};
  std::atomic<int> failed{0};
  std::string fail_msg;
};

namespace knn {

static int upload(DbEngine &D, std::vector<Request *> &batch, std::string &err) {
  const int64_t m = D.db->m;
  const int elem = D.db->dtype == KNN_U8 ? 1 : 4;
  auto ok = [&](hipError_t e, const char *what) {
    if (e != hipSuccess) err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipSuccess;
  };
  static const int32_t minus1 = -1;
  // every host source below (the request's query and descriptor, nq_host)
  // stays valid until the single synchronisation at the end of the batch
  for (Request *r : batch) {
    const int64_t slot = D.submitted % D.qcap;
    QDesc &d = r->dd;
    d = r->d;
    d.q = D.dq + slot * m * elem;
    d.sched = (int32_t)slot;
    d.out_idx = D.didx + slot * kSessionMaxKH;
    d.out_stride = kSessionMaxKH;
    d.out_count = D.dcnt + slot;
    d.out_stats = D.dstats + slot;
    if (!ok(hipMemcpyAsync((void *)d.q, r->q.data(), m * elem, hipMemcpyHostToDevice, D.st), "upload query") ||
        !ok(hipMemcpyAsync(D.E.qd + slot, &d, sizeof(QDesc), hipMemcpyHostToDevice, D.st), "upload desc") ||
        !ok(hipMemcpyAsync(D.E.sched + slot, &r->sc, sizeof(Sched), hipMemcpyHostToDevice, D.st), "upload sched") ||
        !ok(hipMemcpyAsync(D.dcnt + slot, &minus1, sizeof(int32_t), hipMemcpyHostToDevice, D.st), "reset count"))
      return KNN_EDEVICE;
    if (D.db->dtype == KNN_F32) launch_prep_f32(D.E.qd + slot, 1, D.db->n, m, D.db->lo, D.db->hi, D.db->metric, D.st);
    D.ring[slot] = r;
    D.inflight++;
    D.submitted++;
  }
  D.nq_host = D.submitted;
  if (!ok(hipMemcpyAsync(&D.E.ctl->nq, &D.nq_host, sizeof(int32_t), hipMemcpyHostToDevice, D.st), "raise nq") ||
      !ok(hipStreamSynchronize(D.st), "upload sync"))
    return KNN_EDEVICE;
  return KNN_OK;
}

static void fail_all(knn_session_s *S, DbEngine &D, const std::string &msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->fail_msg = msg;
  S->failed = 1;
  for (int64_t s = 0; s < D.qcap; ++s)
    if (D.ring[s]) {
      D.ring[s]->done = true;
      D.ring[s]->err = KNN_EDEVICE;
      D.ring[s] = nullptr;
    }
  D.inflight = 0;
}

static void db_loop(knn_session_s *S, DbEngine *Dp) {
  DbEngine &D = *Dp;
  std::string err;
  while (!S->stop.load()) {
    // 1. admission: move pending requests into free ring entries
    std::vector<Request *> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      int32_t next = D.submitted;
      while (!D.pending.empty() && D.ring[next % D.qcap] == nullptr &&
             D.inflight + (int64_t)batch.size() < D.qcap) {
        batch.push_back(D.pending.front());
        D.pending.pop_front();
        ++next;
      }
      if (batch.empty() && D.inflight == 0) {
        D.cv.wait_for(lk, std::chrono::microseconds(500));
        continue;
      }
    }
    if (!batch.empty() && upload(D, batch, err) != KNN_OK) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->fail_msg = err;
      S->failed = 1;
      for (Request *r : batch) {
        r->done = true;
        r->err = KNN_EDEVICE;
      }
      continue;
    }
    // 2. one round
    engine_step(D.E, true);
    // 3. collect finished queries
    hipError_t e = hipMemcpyAsync(D.hcnt.data(), D.dcnt, sizeof(int32_t) * D.qcap, hipMemcpyDeviceToHost, D.st);
    if (e == hipSuccess) e = hipStreamSynchronize(D.st);
    if (e != hipSuccess) {
      fail_all(S, D, std::string("session step: ") + hipGetErrorString(e));
      continue;
    }
    for (int64_t s = 0; s < D.qcap; ++s) {
      Request *r = D.ring[s];
      if (!r || D.hcnt[s] < 0) continue;
      r->count = D.hcnt[s];
      std::vector<int64_t> idx(std::max<int64_t>(r->d.kh, 1), -1);
      knn_stats st{};
      e = hipMemcpyAsync(idx.data(), D.didx + s * kSessionMaxKH, sizeof(int64_t) * std::min<int64_t>(r->d.kh, kSessionMaxKH),
                         hipMemcpyDeviceToHost, D.st);
      if (e == hipSuccess) e = hipMemcpyAsync(&st, D.dstats + s, sizeof(knn_stats), hipMemcpyDeviceToHost, D.st);
      if (e == hipSuccess) e = hipStreamSynchronize(D.st);
      std::lock_guard<std::mutex> lk(S->mu);
      r->idx.swap(idx);
      r->st = st;
      if (e != hipSuccess) r->err = KNN_EDEVICE;
      r->done = true;
      D.ring[s] = nullptr;
      D.inflight--;
    }
  }
}

}  // namespace knn

using namespace knn;

extern "C" {

int knn_session_create(size_t hbm_budget_bytes, knn_session *out) {
  if (!out) return fail(KNN_EINVAL, "NULL argument");
  if (hbm_budget_bytes < ((size_t)1 << 20)) return fail(KNN_EINVAL, "budget below 1 MiB");
  knn_session_s *S = new knn_session_s();
  S->budget = hbm_budget_bytes;
  *out = S;
  return KNN_OK;
}

int knn_session_add_db(knn_session S, knn_db db, int32_t *db_id) {
  if (!S || !db || !db_id) return fail(KNN_EINVAL, "NULL argument");
  const int64_t n = db->n, m = db->m;
  const int elem = db->dtype == KNN_U8 ? 1 : 4;
  const size_t per_slot = engine_slot_bytes(n, (int32_t)kSessionMaxKH, (int32_t)kSessionMaxKH);
  const size_t per_ring = (size_t)m * elem + kSessionMaxKH * 8 + 4 + sizeof(knn_stats) + sizeof(QDesc) + sizeof(Sched);
  std::unique_ptr<DbEngine> D(new DbEngine());
  D->db = db;
  // Memory admission: each DB reserves half of the budget still free for its
  // query slots (at least one slot); requests beyond its slots wait on the host.
  const size_t avail = S->budget > S->reserved ? S->budget - S->reserved : 0;
  int64_t ns = (int64_t)((avail / 2) / (per_slot + 2 * per_ring));
  ns = std::max<int64_t>(1, std::min<int64_t>(ns, kSessionMaxSlots));
  D->qcap = 2 * ns;
  HIP_TRY(hipStreamCreateWithFlags(&D->st, hipStreamNonBlocking));
  int rc = engine_create(D->E, db, ns, (int32_t)kSessionMaxKH, (int32_t)kSessionMaxKH, D->qcap, D->qcap, D->st, false,
                         false);
  if (rc != KNN_OK) {
    (void)hipStreamDestroy(D->st);
    return rc;
  }
  hipError_t e = hipMalloc(&D->dq, (size_t)D->qcap * m * elem);
  if (e == hipSuccess) e = hipMalloc(&D->didx, sizeof(int64_t) * D->qcap * kSessionMaxKH);
  if (e == hipSuccess) e = hipMalloc(&D->dcnt, sizeof(int32_t) * D->qcap);
  if (e == hipSuccess) e = hipMalloc(&D->dstats, sizeof(knn_stats) * D->qcap);
  Ctl ctl;
  std::memset(&ctl, 0, sizeof(ctl));
  ctl.qcap = (int32_t)D->qcap;
  if (e == hipSuccess) e = hipMemcpyAsync(D->E.ctl, &ctl, sizeof(Ctl), hipMemcpyHostToDevice, D->st);
  if (e == hipSuccess) e = hipStreamSynchronize(D->st);
  if (e != hipSuccess) {
    engine_destroy(D->E);
    (void)hipFree(D->dq);
    (void)hipFree(D->didx);
    (void)hipFree(D->dcnt);
    (void)hipFree(D->dstats);
    (void)hipStreamDestroy(D->st);
    return fail(e == hipErrorOutOfMemory ? KNN_ENOMEM : KNN_EDEVICE, std::string("session add_db: ") + hipGetErrorString(e));
  }
  D->ring.assign(D->qcap, nullptr);
  D->hcnt.assign(D->qcap, -1);
  db->users++;
  std::lock_guard<std::mutex> lk(S->mu);
  S->reserved += (size_t)ns * per_slot + (size_t)D->qcap * per_ring;
  *db_id = (int32_t)S->dbs.size();
  DbEngine *Dp = D.get();
  S->dbs.push_back(std::move(D));
  Dp->worker = std::thread(db_loop, S, Dp);
  return KNN_OK;
}

int knn_session_submit(knn_session S, int32_t db_id, const void *host_query, int32_t k, const knn_params *p,
                       uint64_t *ticket) {
  if (!S || !host_query || !p || !ticket) return fail(KNN_EINVAL, "NULL argument");
  std::unique_ptr<Request> r(new Request());
  knn_db_s *db;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (db_id < 0 || db_id >= (int32_t)S->dbs.size()) return fail(KNN_ENOTFOUND, "unknown db_id");
    db = S->dbs[db_id]->db;
  }
  int rc = make_qdesc(db, k, *p, r->d, r->sc);
  if (rc != KNN_OK) return rc;
  if (r->d.kh > kSessionMaxKH) return fail(KNN_EINVAL, "session requests need k + h <= 512");
  if (S->failed.load()) return fail(KNN_EDEVICE, "session failed: " + S->fail_msg);
  const size_t bytes = (size_t)db->m * (db->dtype == KNN_U8 ? 1 : 4);
  r->q.assign((const uint8_t *)host_query, (const uint8_t *)host_query + bytes);
  r->db_id = db_id;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->dbs[db_id]->pending.push_back(r.get());
    S->reqs.emplace(r->ticket, r.get());
    r.release();
  }
  S->dbs[db_id]->cv.notify_one();
  return KNN_OK;
}

int knn_session_poll(knn_session S, uint64_t ticket, int64_t *host_idx, int32_t *count, knn_stats *st) {
  if (!S) return fail(KNN_EINVAL, "NULL session");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(KNN_ENOTFOUND, "unknown ticket");
  Request *r = it->second;
  if (!r->done) return KNN_PENDING;
  const int err = r->err;
  if (err == KNN_OK) {
    if (host_idx)
      for (int64_t j = 0; j < r->d.kh; ++j) host_idx[j] = j < (int64_t)r->idx.size() ? r->idx[j] : -1;
    if (count) *count = r->count;
    if (st) *st = r->st;
  }
  S->reqs.erase(it);
  delete r;
  if (err != KNN_OK) return fail(err, "request failed: " + S->fail_msg);
  return KNN_OK;
}

int knn_session_destroy(knn_session S) {
  if (!S) return fail(KNN_EINVAL, "NULL session");
  S->stop = true;
  for (auto &up : S->dbs) {
    up->cv.notify_all();
    if (up->worker.joinable()) up->worker.join();
  }
  for (auto &up : S->dbs) {
    DbEngine &D = *up;
    (void)hipStreamSynchronize(D.st);
    engine_destroy(D.E);
    (void)hipFree(D.dq);
    (void)hipFree(D.didx);
    (void)hipFree(D.dcnt);
    (void)hipFree(D.dstats);
    (void)hipStreamDestroy(D.st);
    D.db->users--;
  }
  for (auto &kv : S->reqs) delete kv.second;
  delete S;
  return KNN_OK;
}

}  // extern "C"
