// knn_session.cpp -- serving session: resident DBs, memory-admitted query
// slots, and continuous batching.
//
// Each DB added to a session gets a slot engine (device state for up to
// kSessionMaxSlots in-flight queries, and at most as many as the session's
// budget holds for that DB) on its own HIP stream, device rings for query
// vectors, descriptors and results, and its own worker thread, so that DBs
// progress independently.  Requests of all DBs are admitted against one
// shared budget: a request takes its DB's per-query state bytes (running
// sums, flags, lists and selection space for the DB's n points, plus its
// ring entry) from the budget when it enters a ring entry and returns them
// when its result has been copied out.  A worker loops:
//   1. moves submitted requests into free ring entries while the budget has
//      room for them (uploads the queries, descriptors and schedules of the
//      whole batch, then raises the engine's query count);
//   2. launches one round ("step") on the engine -- queries admitted on the
//      device join at this round boundary while the others continue where
//      they are;
//   3. copies the result counts, then the results of every query that
//      finished in the step, with one synchronisation for each.
// Requests therefore overlap on the device and are admitted as slots and
// memory free up; each result depends only on (query, DB, k, params).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
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
  size_t req_bytes = 0;        // state bytes one request of this DB takes from the budget
  int32_t run_hi = 0;          // 1 + the highest running slot after the last step's admission
  int32_t nq_host = 0;         // source of the query-count upload
  std::condition_variable cv;  // new requests for this DB
  std::thread worker;
};

}  // namespace knn

struct knn_session_s {
  size_t budget = 0;
  size_t in_use = 0;   // state bytes of the requests in ring entries (all DBs)
  std::mutex mu;
  std::vector<std::unique_ptr<knn::DbEngine>> dbs;
  std::unordered_map<uint64_t, knn::Request *> reqs;
  uint64_t next_ticket = 1;
  std::atomic<bool> stop{false};
  std::atomic<int> failed{0};
  std::string fail_msg;
  // KNN_SESSION_FAIL_UPLOAD=j (tests of the failure path): the upload of
  // the session's request number j (counted from 0 over all its DBs) fails
  // as a device copy would, with the batch's earlier requests already in
  // the ring; -1 (unset): never
  int64_t fail_upload = -1;
  std::atomic<int64_t> uploads{0};
};

namespace knn {

static int upload(DbEngine &D, std::vector<Request *> &batch, std::string &err, int64_t fail_at,
                  std::atomic<int64_t> &uploads) {
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
    if (fail_at >= 0 && uploads.fetch_add(1) >= fail_at) {
      err = "upload query: injected failure (KNN_SESSION_FAIL_UPLOAD)";
      return KNN_EDEVICE;
    }
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

// Marks every request of the DB's ring done with an error and frees its
// ring entry and budget (under the session lock); the worker then idles.
static void fail_all(knn_session_s *S, DbEngine &D, const std::string &msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->fail_msg = msg;
  S->failed = 1;
  for (int64_t s = 0; s < D.qcap; ++s)
    if (D.ring[s]) {
      D.ring[s]->done = true;
      D.ring[s]->err = KNN_EDEVICE;
      D.ring[s] = nullptr;
      S->in_use -= D.req_bytes;
    }
  D.inflight = 0;
  for (Request *r : D.pending) {  // never admitted: failed too, so that their polls end
    r->done = true;
    r->err = KNN_EDEVICE;
  }
  D.pending.clear();
}

static void db_loop(knn_session_s *S, DbEngine *Dp) {
  DbEngine &D = *Dp;
  std::string err;
  std::vector<int64_t> fin;  // ring entries whose query finished in this step
  std::vector<std::vector<int64_t>> fidx;
  std::vector<knn_stats> fst;
  while (!S->stop.load()) {
    if (S->failed.load()) {  // a device error: nothing more runs on this session
      std::unique_lock<std::mutex> lk(S->mu);
      D.cv.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    // 1. admission: move pending requests into free ring entries while the
    //    shared budget holds their state
    std::vector<Request *> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      int32_t next = D.submitted;
      while (!D.pending.empty() && D.ring[next % D.qcap] == nullptr &&
             D.inflight + (int64_t)batch.size() < D.qcap && S->in_use + D.req_bytes <= S->budget) {
        batch.push_back(D.pending.front());
        D.pending.pop_front();
        S->in_use += D.req_bytes;
        ++next;
      }
      if (batch.empty() && D.inflight == 0) {
        D.cv.wait_for(lk, std::chrono::microseconds(500));
        continue;
      }
    }
    if (!batch.empty()) {
      const int64_t before = D.submitted;
      if (upload(D, batch, err, S->fail_upload, S->uploads) != KNN_OK) {
        // the requests that reached the ring are failed there; the rest here.
        // Copies already queued read the requests' host queries: wait for
        // them (their own errors aside) before a poll may free a request.
        const int64_t placed = D.submitted - before;
        (void)hipStreamSynchronize(D.st);
        fail_all(S, D, err);
        std::lock_guard<std::mutex> lk(S->mu);
        for (size_t j = (size_t)placed; j < batch.size(); ++j) {
          batch[j]->done = true;
          batch[j]->err = KNN_EDEVICE;
          S->in_use -= D.req_bytes;
        }
        continue;
      }
    }
    // 2. one round over the slots that can be running (admission keeps them
    //    packed below run_hi; new queries are admitted at the end of the step)
    D.E.G.nslots = std::max<int32_t>(1, std::min<int32_t>((int32_t)D.E.ns, D.run_hi));
    engine_step(D.E, true);
    // 3. collect finished queries: the counts (and the new run_hi), then the
    //    rows and statistics of the finished ones, one synchronisation each
    hipError_t e = hipMemcpyAsync(D.hcnt.data(), D.dcnt, sizeof(int32_t) * D.qcap, hipMemcpyDeviceToHost, D.st);
    if (e == hipSuccess) e = hipMemcpyAsync(&D.run_hi, &D.E.ctl->run_hi, sizeof(int32_t), hipMemcpyDeviceToHost, D.st);
    if (e == hipSuccess) e = hipStreamSynchronize(D.st);
    fin.clear();
    for (int64_t s = 0; s < D.qcap && e == hipSuccess; ++s)
      if (D.ring[s] && D.hcnt[s] >= 0) fin.push_back(s);
    if (fidx.size() < fin.size()) fidx.resize(fin.size());
    fst.assign(fin.size(), knn_stats{});
    for (size_t f = 0; f < fin.size() && e == hipSuccess; ++f) {
      const int64_t s = fin[f];
      const int64_t kh = std::max<int64_t>(std::min<int64_t>(D.ring[s]->d.kh, kSessionMaxKH), 1);
      fidx[f].assign(kh, -1);
      e = hipMemcpyAsync(fidx[f].data(), D.didx + s * kSessionMaxKH, sizeof(int64_t) * kh, hipMemcpyDeviceToHost,
                         D.st);
      if (e == hipSuccess) e = hipMemcpyAsync(&fst[f], D.dstats + s, sizeof(knn_stats), hipMemcpyDeviceToHost, D.st);
    }
    if (e == hipSuccess && !fin.empty()) e = hipStreamSynchronize(D.st);
    if (e != hipSuccess) {
      fail_all(S, D, std::string("session step: ") + hipGetErrorString(e));
      continue;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t f = 0; f < fin.size(); ++f) {
      const int64_t s = fin[f];
      Request *r = D.ring[s];
      r->count = D.hcnt[s];
      r->idx.swap(fidx[f]);
      r->st = fst[f];
      r->done = true;
      D.ring[s] = nullptr;
      D.inflight--;
      S->in_use -= D.req_bytes;
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
  if (const char *e = std::getenv("KNN_SESSION_FAIL_UPLOAD")) S->fail_upload = std::atoll(e);
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
  // Slots: as many as the whole budget holds for this DB (a DB may use all
  // of it while the others are idle), at most kSessionMaxSlots; requests
  // beyond the free slots or the free budget wait on the host.
  const size_t req_bytes = per_slot + 2 * per_ring;
  int64_t ns = (int64_t)(S->budget / req_bytes);
  if (ns < 1) return fail(KNN_ENOMEM, "the session budget does not hold one query of this DB");
  ns = std::min<int64_t>(ns, kSessionMaxSlots);
  D->req_bytes = req_bytes;
  D->qcap = 2 * ns;
  HIP_TRY(hipStreamCreateWithFlags(&D->st, hipStreamNonBlocking));
  int rc = engine_create(D->E, db, ns, (int32_t)kSessionMaxKH, (int32_t)kSessionMaxKH, D->qcap, D->qcap, D->st, false,
                         false);
  if (rc != KNN_OK) {
    (void)hipStreamDestroy(D->st);
    return rc;
  }
  D->E.G.packed_admit = 1;  // queries go to the lowest idle slots; steps cover the slots below run_hi
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
  const size_t bytes = (size_t)db->m * (db->dtype == KNN_U8 ? 1 : 4);
  r->q.assign((const uint8_t *)host_query, (const uint8_t *)host_query + bytes);
  r->db_id = db_id;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    // (checked under the lock that a failure is marked under: a request
    // queued after fail_all would never be taken or failed)
    if (S->failed.load()) return fail(KNN_EDEVICE, "session failed: " + S->fail_msg);
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
