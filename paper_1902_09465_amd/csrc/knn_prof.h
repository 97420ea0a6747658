// knn_prof.h -- optional kernel timing for measurement.  When enabled
// (knn_prof_enable), launchers bracket their hot kernels with HIP events on
// the stream they launch on, and kernels add their algorithmic work to
// device counters.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knn {

enum ProfKind {
  PROF_SAMPLE = 0,     // k_sample
  PROF_CAND = 1,       // k_cand_partial + k_cand_merge
  PROF_SELECT = 2,     // k_select_partial + k_select_merge
  PROF_DECIDE = 3,     // k_decide
  PROF_FINISH = 4,     // k_finish
  PROF_NAIVE_GEMM = 5, // naive MFMA scan with fused top-k
  PROF_NAIVE_REST = 6, // naive query prep + merge (+ f32 rescoring)
  PROF_EXACT = 7,      // k_sample launches of a lock-step batch's exact round
  PROF_QL_AUX = 8,     // query-lane sampling: flag transpose + fold of the round totals; or the
                       // gather of a shared coordinate sequence
  PROF_SPARSE = 9,     // point-major batches: per-slot sampling / exact sums of their sparse slots
  PROF_KINDS = 10
};

// Device counters: kProfCopies copies of the four counters, one cache line
// apart.  A block adds to the copy its index selects (device-scope atomics
// on one address serialise); the host sums the copies.
constexpr int kProfCopies = 64, kProfStride = 16;

bool prof_enabled();
uint64_t *prof_device_counters();  // NULL unless enabled
int prof_begin(int kind, hipStream_t st);               // returns a token (or -1)
void prof_end(int token, hipStream_t st, double units); // units: algorithmic work known on the host
void prof_add_host(int idx, uint64_t v);                // host-side counter idx (0..3) += v

}  // namespace knn
