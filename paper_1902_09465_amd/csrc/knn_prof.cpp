// knn_prof.cpp -- event-based kernel timing and work counters (measurement
// support; off by default, no cost when off).
#include "knn_prof.h"

#include <mutex>
#include <string>
#include <vector>

#include "knn_host.h"

namespace knn {

struct ProfRec {
  int kind;
  hipEvent_t a, b;
  double units;
  bool closed;
};

struct ProfState {
  std::mutex mu;
  bool on = false;
  uint64_t *dcnt = nullptr;
  uint64_t host_cnt[4] = {0, 0, 0, 0};  // counters kept on the host ([4..7] of the ABI)
  std::vector<ProfRec> recs;
};

static ProfState &P() {
  static ProfState s;
  return s;
}

bool prof_enabled() { return P().on; }

void prof_add_host(int idx, uint64_t v) {
  ProfState &s = P();
  if (!s.on || idx < 0 || idx > 3) return;
  std::lock_guard<std::mutex> lk(s.mu);
  s.host_cnt[idx] += v;
}
uint64_t *prof_device_counters() { return P().on ? P().dcnt : nullptr; }

int prof_begin(int kind, hipStream_t st) {
  ProfState &s = P();
  if (!s.on) return -1;
  std::lock_guard<std::mutex> lk(s.mu);
  ProfRec r{kind, nullptr, nullptr, 0.0, false};
  // Timing-only events: without the system-scope fence a record does not
  // write back and invalidate the caches, which would slow the next kernel.
  // Kernels on one stream stay ordered by the stream itself.
  const unsigned fl = hipEventDisableSystemFence;
  if (hipEventCreateWithFlags(&r.a, fl) != hipSuccess || hipEventCreateWithFlags(&r.b, fl) != hipSuccess) return -1;
  (void)hipEventRecord(r.a, st);
  s.recs.push_back(r);
  return (int)s.recs.size() - 1;
}

void prof_end(int token, hipStream_t st, double units) {
  ProfState &s = P();
  if (token < 0 || !s.on) return;
  std::lock_guard<std::mutex> lk(s.mu);
  if (token >= (int)s.recs.size()) return;
  (void)hipEventRecord(s.recs[token].b, st);
  s.recs[token].units = units;
  s.recs[token].closed = true;
}

static void clear_locked(ProfState &s) {
  for (auto &r : s.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  s.recs.clear();
}

}  // namespace knn

using namespace knn;

extern "C" {

int knn_prof_enable(int on) {
  ProfState &s = P();
  std::lock_guard<std::mutex> lk(s.mu);
  clear_locked(s);
  const size_t words = (size_t)kProfCopies * kProfStride;
  if (on && !s.dcnt) HIP_TRY(hipMalloc(&s.dcnt, sizeof(uint64_t) * words));
  if (s.dcnt) HIP_TRY(hipMemset(s.dcnt, 0, sizeof(uint64_t) * words));
  s.host_cnt[0] = s.host_cnt[1] = s.host_cnt[2] = s.host_cnt[3] = 0;
  s.on = on != 0;
  return KNN_OK;
}

int knn_prof_read(int32_t kind, double *total_ms, int64_t *launches, double *units) {
  ProfState &s = P();
  std::lock_guard<std::mutex> lk(s.mu);
  double ms = 0.0, u = 0.0;
  int64_t cnt = 0;
  for (auto &r : s.recs) {
    if (r.kind != kind || !r.closed) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(KNN_EDEVICE, "event sync");
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(KNN_EDEVICE, "event time");
    ms += t;
    u += r.units;
    ++cnt;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = cnt;
  if (units) *units = u;
  return KNN_OK;
}

int knn_prof_counters(uint64_t *host_out8) {
  ProfState &s = P();
  if (!host_out8) return fail(KNN_EINVAL, "NULL argument");
  for (int i = 0; i < 8; ++i) host_out8[i] = 0;
  if (!s.dcnt) return KNN_OK;
  HIP_TRY(hipDeviceSynchronize());
  std::vector<uint64_t> all((size_t)kProfCopies * kProfStride);
  HIP_TRY(hipMemcpy(all.data(), s.dcnt, sizeof(uint64_t) * all.size(), hipMemcpyDeviceToHost));
  for (int c = 0; c < kProfCopies; ++c)
    for (int i = 0; i < 4; ++i) host_out8[i] += all[(size_t)c * kProfStride + i];
  std::lock_guard<std::mutex> lk(s.mu);
  for (int i = 0; i < 4; ++i) host_out8[4 + i] = s.host_cnt[i];
  return KNN_OK;
}

}  // extern "C"
