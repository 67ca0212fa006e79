// Per-thread kernel timing with HIP events (ap_profile_enable / ap_profile_read).
#include <hip/hip_runtime.h>

#include <vector>

#include "apsort.h"
#include "apsort_internal.h"

namespace aps {

struct PendingLaunch {
  int kind;
  hipEvent_t start, stop;
};

struct ProfState {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<PendingLaunch> pending;
  int open_kind = -1;
  hipEvent_t open_start = nullptr;
  double ms[AP_NKINDS] = {};
  uint64_t launches[AP_NKINDS] = {};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~ProfState() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

static thread_local ProfState t_prof;

bool prof_active() { return t_prof.on; }

void prof_begin(int kind, hipStream_t s) {
  ProfState& p = t_prof;
  if (!p.on) return;
  p.open_kind = kind;
  p.open_start = p.get();
  if (p.open_start) (void)hipEventRecord(p.open_start, s);
}

void prof_end(hipStream_t s) {
  ProfState& p = t_prof;
  if (!p.on || p.open_kind < 0 || !p.open_start) return;
  hipEvent_t stop = p.get();
  if (!stop) return;
  (void)hipEventRecord(stop, s);
  p.pending.push_back({p.open_kind, p.open_start, stop});
  p.open_kind = -1;
  p.open_start = nullptr;
}

}  // namespace aps

using namespace aps;

extern "C" {

ap_status ap_profile_enable(int on) {
  t_prof.on = on != 0;
  return AP_OK;
}

ap_status ap_profile_read(double* ms, uint64_t* launches, int nkinds) {
  if (!ms || !launches || nkinds < AP_NKINDS) return fail(AP_ERR_INVALID, "need AP_NKINDS entries");
  ProfState& p = t_prof;
  for (auto& l : p.pending) {
    hipError_t e = hipEventSynchronize(l.stop);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float t = 0.f;
    e = hipEventElapsedTime(&t, l.start, l.stop);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    if (l.kind >= 0 && l.kind < AP_NKINDS) {
      p.ms[l.kind] += t;
      p.launches[l.kind] += 1;
    }
    p.pool.push_back(l.start);
    p.pool.push_back(l.stop);
  }
  p.pending.clear();
  for (int k = 0; k < AP_NKINDS; ++k) {
    ms[k] = p.ms[k];
    launches[k] = p.launches[k];
    p.ms[k] = 0.0;
    p.launches[k] = 0;
  }
  return AP_OK;
}

}  // extern "C"
