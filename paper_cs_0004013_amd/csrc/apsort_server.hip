// HIP executor and C entry points of the sort-request server (ap_server_*).
//
// Each slot owns a non-blocking stream, a completion event and a small header on the device (the
// segmented-sort control block, the descriptor array, and the device-wide sort's control words,
// which are zeroed once and left zero by every sort).  Scratch comes from one arena of the
// memory budget, shared by the slots through the core's ledger.  A batch of short requests
// becomes one launch of the persistent segmented kernel over host-built descriptors (longest
// first), each descriptor pointing at the caller's input and output buffers directly, so no key is
// copied in or out.  A long request runs alone through the device-wide sort with its reserved
// range of the arena as its workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "apsort.h"
#include "apsort_internal.h"
#include "apsort_seg_types.h"
#include "apsort_server_core.h"

namespace aps {

static size_t up256s(size_t x) { return (x + 255) / 256 * 256; }

class HipExecutor : public srv::Executor {
 public:
  struct SlotRes {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    char* header = nullptr;  // [control block][descriptor array][sort control] on the device
    SegDesc* h_desc = nullptr;
    SegCtl* ctl = nullptr;
    SegDesc* d_desc = nullptr;
    char* sort_ctl = nullptr;  // [0, init_bytes) of the device-wide sort's workspace layout
  };

  ap_status init(int nslots, size_t budget, int max_batch) {
    if (hipGetDevice(&dev_) != hipSuccess) return fail(AP_ERR_HIP, "hipGetDevice failed");
    tile_ = 2048;  // smallest tile of any configuration: longer requests get scratch
    max_batch_ = max_batch;
    const size_t sort_ctl = up256s(layout_for(0).init_bytes);
    const size_t header = up256s(sizeof(SegCtl)) + up256s(sizeof(SegDesc) * (size_t)max_batch) + sort_ctl;
    budget_ = budget / 256 * 256;
    if (budget_ < 256) return fail(AP_ERR_BUDGET, "budget below the minimum of 256 bytes");
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&arena_), budget_);
    if (e != hipSuccess) return hip_fail(e, "server scratch arena allocation");
    slots_.resize(nslots);
    for (auto& sl : slots_) {
      e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sl.header), header);
      if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_desc), sizeof(SegDesc) * max_batch);
      if (e != hipSuccess) return hip_fail(e, "server slot allocation");
      sl.ctl = reinterpret_cast<SegCtl*>(sl.header);
      sl.d_desc = reinterpret_cast<SegDesc*>(sl.header + up256s(sizeof(SegCtl)));
      sl.sort_ctl = sl.header + (header - sort_ctl);
      ap_status st = fill_u32(reinterpret_cast<uint32_t*>(sl.ctl), 0u, up256s(sizeof(SegCtl)) / 4, sl.stream);
      if (st == AP_OK) st = fill_u32(reinterpret_cast<uint32_t*>(sl.sort_ctl), 0u, sort_ctl / 4, sl.stream);
      if (st != AP_OK) return st;
    }
    ap_status st = check_lane_order(slots_[0].stream);
    if (st != AP_OK) return st;
    for (auto& sl : slots_) {
      hipError_t e = hipStreamSynchronize(sl.stream);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    return AP_OK;
  }

  ~HipExecutor() override {
    for (auto& sl : slots_) {
      if (sl.stream) (void)hipStreamSynchronize(sl.stream);
      if (sl.h_desc) (void)hipHostFree(sl.h_desc);
      if (sl.header) (void)hipFree(sl.header);
      if (sl.ev) (void)hipEventDestroy(sl.ev);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (arena_) (void)hipFree(arena_);
  }

  int num_slots() const override { return (int)slots_.size(); }
  size_t scratch_budget() const override { return budget_; }

  size_t scratch_bytes(const srv::Request& r, bool alone) const override {
    if (alone) {
      const Layout L = layout_for(r.n);
      return L.total - L.tctr;  // the control words live in the slot's header
    }
    return r.n > tile_ ? up256s(r.n * sizeof(uint32_t)) : 0;  // one-tile requests need no scratch
  }

  void thread_init() override { (void)hipSetDevice(dev_); }

  ap_status launch_batch(int slot, std::vector<srv::Request*>& reqs, size_t scratch_off, size_t) override {
    ApRange range("ap_server batch");
    SlotRes& sl = slots_[slot];
    // A batch of one request short enough for one workgroup (what a lightly loaded server forms):
    // the single-array sort's one launch, with no descriptor upload.
    if (reqs.size() == 1 && reqs[0]->n >= 1 && reqs[0]->n <= kSmallSortMax) {
      srv::Request* r = reqs[0];
      const ap_status st = enqueue_small_sort(r->in, r->out, r->n, r->P, r->P > 1 ? r->spl : nullptr, sl.stream);
      if (st != AP_OK) return st;
      const hipError_t e = hipEventRecord(sl.ev, sl.stream);
      return e == hipSuccess ? AP_OK : hip_fail(e, "hipEventRecord");
    }
    char* const scratch = arena_ + scratch_off;
    std::sort(reqs.begin(), reqs.end(), [](const srv::Request* a, const srv::Request* b) { return a->n > b->n; });
    size_t used = 0;
    uint32_t cnt = 0;
    for (srv::Request* r : reqs) {
      SegDesc& d = sl.h_desc[cnt++];
      d.src = r->in;
      d.dst = r->out;
      d.tmp = nullptr;
      if (r->n > tile_) {
        d.tmp = reinterpret_cast<uint32_t*>(scratch + used);
        used += up256s(r->n * sizeof(uint32_t));
      }
      d.spl = r->P > 1 ? r->spl : nullptr;
      d.n = (uint32_t)r->n;
      d.P = (uint32_t)r->P;
      d.pad[0] = d.pad[1] = 0u;
    }
    hipError_t e = hipMemcpyAsync(sl.d_desc, sl.h_desc, sizeof(SegDesc) * cnt, hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    // The descriptors are sorted longest first, so each length group is a contiguous item range
    // (lengths 0 and 1 count as class 1).
    SegGroup grp[kSegGroups];
    seg_groups(grp);
    ap_status gst = seg_groups_check(grp);
    if (gst != AP_OK) return gst;
    for (int g = 0; g < kSegGroups; ++g) {
      if (grp[g].cls_lo > grp[g].cls_hi) continue;
      uint32_t lo = cnt, hi = 0;
      for (uint32_t i = 0; i < cnt; ++i) {
        const uint32_t n = sl.h_desc[i].n;
        const int c = n < 2 ? 1 : 32 - __builtin_clz(n - 1u);  // ceil(log2(n)), as on the device
        if (c >= grp[g].cls_lo && c <= grp[g].cls_hi) {
          lo = std::min(lo, i);
          hi = i + 1;
        }
      }
      if (lo >= hi) continue;
      launch_seg_group(grp[g], dim3(seg_workgroups(grp[g], hi - lo)), sl.stream, sl.d_desc, lo, hi, g, sl.ctl);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_seg_sort");
    e = hipEventRecord(sl.ev, sl.stream);
    return e == hipSuccess ? AP_OK : hip_fail(e, "hipEventRecord");
  }

  ap_status launch_alone(int slot, srv::Request* r, size_t scratch_off, size_t scratch_len) override {
    SlotRes& sl = slots_[slot];
    char* const scratch = arena_ + scratch_off;
    const Layout L = layout_for(r->n);
    // The layout depends on the pass tile shape, a process-wide setting (ap_set_pass_shape): if it
    // changed since the request was admitted, the reserved range may no longer hold the layout.
    if (r->n && L.total - L.tctr > scratch_len)
      return fail(AP_ERR_INVALID, "pass shape changed after the request was admitted: its scratch no longer fits");
    ap_status st = AP_OK;
    if (r->n == 0) {
      if (r->P > 1 && r->spl) st = fill_u32(r->spl, 0xFFFFFFFFu, (size_t)r->P - 1, sl.stream);
    } else {
      st = enqueue_sort_parts(r->in, r->out, r->n, r->P, r->P > 1 ? r->spl : nullptr, sl.sort_ctl, scratch, L,
                              sl.stream);
    }
    if (st != AP_OK) return st;
    hipError_t e = hipEventRecord(sl.ev, sl.stream);
    return e == hipSuccess ? AP_OK : hip_fail(e, "hipEventRecord");
  }

  int query(int slot) override {
    const hipError_t e = hipEventQuery(slots_[slot].ev);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return -1;
  }

 private:
  int dev_ = 0;
  size_t tile_ = 8192;
  int max_batch_ = 256;
  size_t budget_ = 0;
  char* arena_ = nullptr;  // the scratch arena, budget_ bytes
  std::vector<SlotRes> slots_;
};

}  // namespace aps

struct ap_server {
  aps::HipExecutor* ex;
  aps::srv::Server* core;
};

using namespace aps;

// Nearest-rank percentile of a sorted, non-empty sample.
static double sorted_pct(const std::vector<double>& v, double p) {
  const double r = std::ceil(p * (double)v.size());
  const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::max(0.0, r - 1.0));
  return v[i];
}

extern "C" {

ap_status ap_server_create(const ap_server_cfg* cfg, ap_server** out) {
  if (!out) return fail(AP_ERR_INVALID, "out is NULL");
  *out = nullptr;
  srv::Config c;
  if (cfg) {
    if (cfg->hbm_budget_bytes) c.budget = cfg->hbm_budget_bytes;
    if (cfg->num_streams > 0) c.num_streams = cfg->num_streams;
    if (cfg->max_batch > 0) c.max_batch = cfg->max_batch;
    if (cfg->max_queue > 0) c.max_queue = cfg->max_queue;
    if (cfg->alone_min_keys) c.alone_min_keys = cfg->alone_min_keys;
  }
  if (c.num_streams > 64 || c.max_batch > (1 << 20)) return fail(AP_ERR_INVALID, "server configuration out of range");
  HipExecutor* ex = new HipExecutor();
  ap_status st = ex->init(c.num_streams, c.budget, c.max_batch);
  if (st != AP_OK) {
    delete ex;
    return st;
  }
  ap_server* s = new ap_server{ex, new srv::Server(c, ex)};
  *out = s;
  return AP_OK;
}

ap_status ap_server_submit(ap_server* s, const uint32_t* d_in, uint32_t* d_out, size_t n, int P,
                           uint32_t* d_splitters, uint64_t* ticket) {
  if (!s) return fail(AP_ERR_INVALID, "server is NULL");
  const ap_status st = s->core->submit(d_in, d_out, n, P, d_splitters, 0u, ticket);
  return st == AP_OK ? st : fail(st, "ap_server_submit rejected the request (status %d)", (int)st);
}

ap_status ap_server_submit_flags(ap_server* s, const uint32_t* d_in, uint32_t* d_out, size_t n, int P,
                                 uint32_t* d_splitters, unsigned flags, uint64_t* ticket) {
  if (!s) return fail(AP_ERR_INVALID, "server is NULL");
  const ap_status st = s->core->submit(d_in, d_out, n, P, d_splitters, flags, ticket);
  return st == AP_OK ? st : fail(st, "ap_server_submit rejected the request (status %d)", (int)st);
}

ap_status ap_server_submit_at(ap_server* s, const uint32_t* d_in, uint32_t* d_out, size_t n, int P,
                              uint32_t* d_splitters, unsigned flags, uint64_t arrival_ns, uint64_t* ticket) {
  if (!s) return fail(AP_ERR_INVALID, "server is NULL");
  const ap_status st = s->core->submit(d_in, d_out, n, P, d_splitters, flags, ticket, arrival_ns);
  return st == AP_OK ? st : fail(st, "ap_server_submit rejected the request (status %d)", (int)st);
}

ap_status ap_server_wait(ap_server* s, uint64_t ticket, int64_t timeout_us) {
  if (!s) return fail(AP_ERR_INVALID, "server is NULL");
  return s->core->wait(ticket, timeout_us);
}

ap_status ap_server_poll(ap_server* s, uint64_t ticket) {
  if (!s) return fail(AP_ERR_INVALID, "server is NULL");
  return s->core->poll(ticket);
}

ap_status ap_server_get_stats(ap_server* s, ap_server_stats* out, int reset_latencies) {
  if (!s || !out) return fail(AP_ERR_INVALID, "NULL argument");
  srv::Stats st = s->core->stats();
  std::memset(out, 0, sizeof *out);
  out->submitted = st.submitted;
  out->completed = st.completed;
  out->failed = st.failed;
  out->cancelled = st.cancelled;
  out->batches = st.batches;
  out->alone = st.alone;
  out->keys = st.keys;
  std::vector<double>& v = st.latency_us;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    double sum = 0;
    for (double x : v) sum += x;
    out->p50_us = sorted_pct(v, 0.50);
    out->p99_us = sorted_pct(v, 0.99);
    out->mean_us = sum / (double)v.size();
    out->max_us = v.back();
    out->latency_samples = v.size();
  }
  std::vector<double>& q = st.queue_us;
  if (!q.empty()) {
    std::sort(q.begin(), q.end());
    out->queue_p50_us = sorted_pct(q, 0.50);
    out->queue_p99_us = sorted_pct(q, 0.99);
  }
  out->scratch_budget_bytes = st.scratch_total;
  out->scratch_peak_bytes = st.scratch_peak;
  if (reset_latencies) s->core->reset_latencies();
  return AP_OK;
}

ap_status ap_server_destroy(ap_server* s) {
  if (!s) return fail(AP_ERR_INVALID, "server is NULL");
  s->core->shutdown();
  delete s->core;
  delete s->ex;
  delete s;
  return AP_OK;
}

}  // extern "C"
