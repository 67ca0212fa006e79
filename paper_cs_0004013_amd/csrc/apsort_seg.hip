// Host side of the batched segmented sort (ap_sort_u32_segmented): workspace, launch sequence and
// hipGraph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "apsort.h"
#include "apsort_internal.h"
#include "apsort_seg_kernels.h"

namespace aps {

// Kernel configurations selectable per length group (see seg_config_for).
struct SegCfg {
  int bits, waves, ipt;
};
static const SegCfg kSegCfgs[] = {
    {8, 8, 16},   // 0: 512 threads, 8192-key tiles (default for every group)
    {8, 16, 8},   // 1: 1024 threads, 8192-key tiles
    {8, 4, 16},   // 2: 256 threads, 4096-key tiles
    {8, 4, 8},    // 3: 256 threads, 2048-key tiles
    {4, 4, 8},    // 4: 4-bit digits, 256 threads, 2048-key tiles
    {8, 8, 8},    // 5: 512 threads, 4096-key tiles
    {6, 4, 8},    // 6: 6-bit digits, 256 threads, 2048-key tiles
};
constexpr int kNumSegCfgs = sizeof(kSegCfgs) / sizeof(kSegCfgs[0]);

template <int BITS>
constexpr int seg_lcopies() {
  constexpr int hw = ((32 + BITS - 1) / BITS) << BITS;
  constexpr int c = 15360 / (hw + 1);
  return c < 1 ? 1 : (c > 15 ? 15 : c);
}

template <int BITS, int WAVES, int IPT>
static void launch_seg_sort(dim3 grid, hipStream_t s, const SegDesc* order, uint32_t nwork, SegCtl* ctl) {
  hipLaunchKernelGGL((k_seg_sort<BITS, WAVES, IPT, seg_lcopies<BITS>()>), grid, dim3(WAVES * 64), 0, s, order,
                     nwork, ctl);
}

void launch_seg_cfg(int cfg, dim3 grid, hipStream_t s, const SegDesc* order, uint32_t nwork, SegCtl* ctl) {
  switch (cfg) {
    case 1: launch_seg_sort<8, 16, 8>(grid, s, order, nwork, ctl); break;
    case 2: launch_seg_sort<8, 4, 16>(grid, s, order, nwork, ctl); break;
    case 3: launch_seg_sort<8, 4, 8>(grid, s, order, nwork, ctl); break;
    case 4: launch_seg_sort<4, 4, 8>(grid, s, order, nwork, ctl); break;
    case 5: launch_seg_sort<8, 8, 8>(grid, s, order, nwork, ctl); break;
    case 6: launch_seg_sort<6, 4, 8>(grid, s, order, nwork, ctl); break;
    default: launch_seg_sort<8, 8, 16>(grid, s, order, nwork, ctl); break;
  }
}

int seg_workgroups(int cfg, uint32_t nwork) {
  const int per_cu = (kSegCfgs[cfg].waves * 64 >= 1024) ? 1 : 2;
  return (int)std::max<uint32_t>(1u, std::min<uint32_t>(nwork, (uint32_t)(per_cu * device_cus())));
}

int seg_tile_keys(int cfg) { return kSegCfgs[cfg].waves * 64 * kSegCfgs[cfg].ipt; }

static int g_seg_cfg = 0;  // configuration of the persistent kernel (set by the tuner)
int seg_config() { return g_seg_cfg; }

// Workspace: [SegCtl | pad to 256][order: nseg descriptors | pad][tmp n_total u32]
struct SegLayout {
  size_t ctl, order, tmp, total;
};
static size_t up256(size_t x) { return (x + 255) / 256 * 256; }
static SegLayout seg_layout(size_t n_total, int nseg) {
  SegLayout L{};
  size_t off = 0;
  L.ctl = off;   off += up256(sizeof(SegCtl));
  L.order = off; off += up256(sizeof(SegDesc) * (size_t)std::max(nseg, 1));
  L.tmp = off;   off += up256(sizeof(uint32_t) * std::max<size_t>(n_total, 1));
  L.total = off;
  return L;
}

// ---------------------------------------------------------------- workspace + graph cache
struct SegEntry {
  int dev;
  hipStream_t stream;
  void* ws;
  size_t bytes;
  // graph replay key
  hipGraphExec_t exec;
  const void* k_keys;
  size_t k_n;
  const void* k_off;
  int k_nseg;
  const void* k_status;
  int k_cfg;
};
static std::mutex g_seg_mu;
static std::vector<SegEntry> g_seg;

static ap_status seg_entry(hipStream_t s, size_t need, SegEntry** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  ap_status st = check_lane_order(s);
  if (st != AP_OK) return st;
  for (auto& c : g_seg) {
    if (c.dev != dev || c.stream != s) continue;
    if (c.bytes < need) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      if (c.exec) (void)hipGraphExecDestroy(c.exec);
      c.exec = nullptr;
      (void)hipFree(c.ws);
      c.ws = nullptr;
      c.bytes = 0;
      const size_t bytes = std::max(need, c.bytes + c.bytes / 4);
      e = hipMalloc(&c.ws, bytes);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc(segmented workspace)");
      c.bytes = bytes;
      st = fill_u32(static_cast<uint32_t*>(c.ws), 0u, up256(sizeof(SegCtl)) / 4, s);
      if (st != AP_OK) return st;
    }
    *out = &c;
    return AP_OK;
  }
  SegEntry c{};
  c.dev = dev;
  c.stream = s;
  e = hipMalloc(&c.ws, need);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(segmented workspace)");
  c.bytes = need;
  st = fill_u32(static_cast<uint32_t*>(c.ws), 0u, up256(sizeof(SegCtl)) / 4, s);
  if (st != AP_OK) {
    (void)hipFree(c.ws);
    return st;
  }
  g_seg.push_back(c);
  *out = &g_seg.back();
  return AP_OK;
}

// The launch sequence: classify -> fill -> persistent sort.  No host synchronisation; every grid
// size is fixed by (nseg, device), so the sequence can be captured once and replayed.
ap_status enqueue_segmented(uint32_t* d_keys, size_t n_total, const uint32_t* d_off, int nseg, uint32_t* d_status,
                            void* ws, const SegLayout& L, int cfg, hipStream_t s) {
  char* w = static_cast<char*>(ws);
  SegCtl* ctl = reinterpret_cast<SegCtl*>(w + L.ctl);
  SegDesc* order = reinterpret_cast<SegDesc*>(w + L.order);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(w + L.tmp);
  const int cus = device_cus();
  const uint32_t g1 = (uint32_t)std::min<int>((nseg + 255) / 256 + 1, 4 * cus);
  prof_begin(AP_KIND_SEG, s);
  hipLaunchKernelGGL(k_seg_classify, dim3(g1), dim3(256), 0, s, d_off, (uint32_t)nseg, (uint32_t)n_total, ctl,
                     d_status);
  hipLaunchKernelGGL(k_seg_fill, dim3(g1), dim3(256), 0, s, d_off, (uint32_t)nseg, (uint32_t)n_total, ctl, d_keys,
                     tmp, order);
  launch_seg_cfg(cfg, dim3(seg_workgroups(cfg, (uint32_t)nseg)), s, order, ~0u, ctl);
  prof_end(s);
  return check_launch(s, "k_seg_sort");
}

}  // namespace aps

using namespace aps;

extern "C" {

ap_status ap_sort_u32_segmented(uint32_t* d_keys, size_t n_total, const uint32_t* d_offsets, int nseg,
                                uint32_t* d_status, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (nseg < 0) return fail(AP_ERR_INVALID, "nseg must be >= 0");
  if (n_total >= AP_MAX_KEYS) return fail(AP_ERR_INVALID, "n_total must be < 2^30");
  if (nseg == 0) return d_status ? fill_u32(d_status, 0u, 1, s) : AP_OK;
  if (!d_offsets) return fail(AP_ERR_INVALID, "d_offsets is NULL");
  if (n_total && !d_keys) return fail(AP_ERR_INVALID, "d_keys is NULL with n_total > 0");
  if (((uintptr_t)d_keys | (uintptr_t)d_offsets) & 3u) return fail(AP_ERR_INVALID, "pointers must be 4-byte aligned");
  const SegLayout L = seg_layout(n_total, nseg);
  std::lock_guard<std::mutex> lk(g_seg_mu);
  SegEntry* ent = nullptr;
  ap_status st = seg_entry(s, L.total, &ent);
  if (st != AP_OK) return st;
  const int cfg = g_seg_cfg;

  // Replay a captured graph when the call repeats the previous one on this stream; capture
  // otherwise (only on a non-default stream that is not itself being captured).
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (s) {
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  }
  const bool graphable = s != nullptr && cap == hipStreamCaptureStatusNone && !prof_active();
  if (!graphable) return enqueue_segmented(d_keys, n_total, d_offsets, nseg, d_status, ent->ws, L, cfg, s);
  const bool same = ent->exec && ent->k_keys == d_keys && ent->k_n == n_total && ent->k_off == d_offsets &&
                    ent->k_nseg == nseg && ent->k_status == d_status && ent->k_cfg == cfg;
  if (!same) {
    if (ent->exec) {
      (void)hipGraphExecDestroy(ent->exec);
      ent->exec = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    st = enqueue_segmented(d_keys, n_total, d_offsets, nseg, d_status, ent->ws, L, cfg, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st != AP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&ent->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      ent->exec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    ent->k_keys = d_keys;
    ent->k_n = n_total;
    ent->k_off = d_offsets;
    ent->k_nseg = nseg;
    ent->k_status = d_status;
    ent->k_cfg = cfg;
  }
  hipError_t e = hipGraphLaunch(ent->exec, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return AP_OK;
}

size_t ap_segmented_workspace_bytes(size_t n_total, int nseg) {
  if (n_total >= AP_MAX_KEYS || nseg < 0) return 0;
  return seg_layout(n_total, nseg).total;
}

ap_status ap_segmented_set_config(int cfg) {
  if (cfg < 0 || cfg >= kNumSegCfgs) return fail(AP_ERR_INVALID, "config index out of range");
  g_seg_cfg = cfg;
  return AP_OK;
}

int ap_segmented_num_configs(void) { return kNumSegCfgs; }

}  // extern "C"
