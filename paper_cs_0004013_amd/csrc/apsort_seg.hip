// Host side of the batched segmented sort (ap_sort_u32_segmented): workspace, launch sequence and
// hipGraph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "apsort.h"
#include "apsort_internal.h"
#include "apsort_seg_kernels.h"
#include "apsort_seg_long.h"

namespace aps {

// Kernel configurations selectable per length group (see seg_config_for).
struct SegCfg {
  int bits, waves, ipt;
};
static const SegCfg kSegCfgs[] = {
    {8, 8, 16},   // 0: 512 threads, 8192-key tiles
    {8, 16, 8},   // 1: 1024 threads, 8192-key tiles
    {8, 4, 16},   // 2: 256 threads, 4096-key tiles
    {8, 4, 8},    // 3: 256 threads, 2048-key tiles
    {4, 4, 8},    // 4: 4-bit digits, 256 threads, 2048-key tiles
    {8, 8, 8},    // 5: 512 threads, 4096-key tiles
    {6, 4, 8},    // 6: 6-bit digits, 256 threads, 2048-key tiles
    {10, 4, 8},   // 7: 10-bit digits (4 sweeps, 1024 buckets), 256 threads, 2048-key tiles
    {11, 4, 8},   // 8: 11-bit digits (3 sweeps, 2048 buckets), 256 threads, 2048-key tiles
    {11, 8, 16},  // 9: 11-bit digits, 512 threads, 8192-key tiles
    {8, 16, 16},  // 10: 1024 threads, 16384-key tiles (segments up to 16K keys in one tile)
    {8, 8, 32},   // 11: 512 threads, 16384-key tiles
};
constexpr int kNumSegCfgs = sizeof(kSegCfgs) / sizeof(kSegCfgs[0]);

template <int BITS>
constexpr int seg_lcopies() {
  constexpr int hw = ((32 + BITS - 1) / BITS) << BITS;
  constexpr int c = 15360 / (hw + 1);
  return c < 1 ? 1 : (c > 15 ? 15 : c);
}

// The rank with lane-ordered LDS atomics only on a device that passed the lane-order check
// (lane_order_ok(), also false while the mask rank is forced by ap_set_rank_mode(1)); the ballot
// rank otherwise.  A group whose segments all fit one tile never runs the histogram sweep of
// longer segments, so it is built with a single histogram copy: its workgroup then needs a
// fraction of the LDS (19 instead of 63 KiB for 2048-key tiles), which leaves room on a CU for
// the workgroups of the groups running beside it.
template <int BITS, int WAVES, int IPT>
static void launch_seg_sort(bool one_tile, dim3 grid, hipStream_t s, const SegDesc* order, uint32_t lo, uint32_t hi,
                            int cls_lo, int cls_hi, int grp, SegCtl* ctl) {
  constexpr int LC = seg_lcopies<BITS>();
  if (one_tile) {
    if (lane_order_ok())
      hipLaunchKernelGGL((k_seg_sort<BITS, WAVES, IPT, 1, SEG_RANK_ATOMIC>), grid, dim3(WAVES * 64), 0, s, order, lo,
                         hi, cls_lo, cls_hi, grp, ctl);
    else
      hipLaunchKernelGGL((k_seg_sort<BITS, WAVES, IPT, 1, SEG_RANK_BALLOT>), grid, dim3(WAVES * 64), 0, s, order, lo,
                         hi, cls_lo, cls_hi, grp, ctl);
    return;
  }
  if (lane_order_ok())
    hipLaunchKernelGGL((k_seg_sort<BITS, WAVES, IPT, LC, SEG_RANK_ATOMIC>), grid, dim3(WAVES * 64), 0, s, order, lo, hi,
                       cls_lo, cls_hi, grp, ctl);
  else
    hipLaunchKernelGGL((k_seg_sort<BITS, WAVES, IPT, LC, SEG_RANK_BALLOT>), grid, dim3(WAVES * 64), 0, s, order, lo, hi,
                       cls_lo, cls_hi, grp, ctl);
}

// Every segment of the group fits one tile of its configuration: the longest length of class c
// is 2^c keys.
bool seg_group_one_tile(const SegGroup& g) {
  return g.cls_hi <= 30 && ((size_t)1 << g.cls_hi) <= (size_t)seg_tile_keys(g.cfg);
}

// One persistent kernel of the group's configuration over work items [lo, hi) (or, with
// hi == ~0u, over the device-built work order's length classes of the group), taking items from
// head[grp].
void launch_seg_group(const SegGroup& g, dim3 grid, hipStream_t s, const SegDesc* order, uint32_t lo, uint32_t hi,
                      int grp, SegCtl* ctl) {
  const bool ot = seg_group_one_tile(g);
  const int a = g.cls_lo, b = g.cls_hi;
  switch (g.cfg) {
    case 1: launch_seg_sort<8, 16, 8>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 2: launch_seg_sort<8, 4, 16>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 3: launch_seg_sort<8, 4, 8>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 4: launch_seg_sort<4, 4, 8>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 5: launch_seg_sort<8, 8, 8>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 6: launch_seg_sort<6, 4, 8>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 7: launch_seg_sort<10, 4, 8>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 8: launch_seg_sort<11, 4, 8>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 9: launch_seg_sort<11, 8, 16>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 10: launch_seg_sort<8, 16, 16>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    case 11: launch_seg_sort<8, 8, 32>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
    default: launch_seg_sort<8, 8, 16>(ot, grid, s, order, lo, hi, a, b, grp, ctl); break;
  }
}

// LDS of one workgroup of each configuration (the kernel's only shared object).
template <int BITS, int WAVES, int IPT>
constexpr size_t seg_lds() {
  return sizeof(SegSmem<BITS, WAVES, IPT, seg_lcopies<BITS>()>);
}
static size_t seg_cfg_lds(int cfg) {
  switch (cfg) {
    case 1: return seg_lds<8, 16, 8>();
    case 2: return seg_lds<8, 4, 16>();
    case 3: return seg_lds<8, 4, 8>();
    case 4: return seg_lds<4, 4, 8>();
    case 5: return seg_lds<8, 8, 8>();
    case 6: return seg_lds<6, 4, 8>();
    case 7: return seg_lds<10, 4, 8>();
    case 8: return seg_lds<11, 4, 8>();
    case 9: return seg_lds<11, 8, 16>();
    case 10: return seg_lds<8, 16, 16>();
    case 11: return seg_lds<8, 8, 32>();
    default: return seg_lds<8, 8, 16>();
  }
}

// Persistent grid: as many workgroups as fit on the device at once (by threads: two workgroups of
// up to 512 threads per CU, one of 1024; and by the 160 KiB of LDS per CU of the build with every
// histogram copy), at most one per work item.  One-tile groups keep this grid although their
// build needs less LDS: a larger grid for them measured slower on the mixed batches (1-1.3%), as
// their extra workgroups crowd the CUs that the longer segments' group runs on, while the smaller
// LDS alone lets the groups' workgroups share CUs better (the bucketing sort's local sorts, 2^15
// buckets of ~2K keys: 1.04 -> 0.99 ms per sort).
int seg_workgroups(const SegGroup& g, uint32_t nwork) {
  const int waves = kSegCfgs[g.cfg].waves;
  int per_cu = waves * 64 >= 1024 ? 1 : (waves <= 4 ? 4 : 2);
  per_cu = std::max(1, std::min(per_cu, (int)((size_t)160 * 1024 / seg_cfg_lds(g.cfg))));
  return (int)std::max<uint32_t>(1u, std::min<uint32_t>(nwork, (uint32_t)(per_cu * device_cus())));
}

int seg_tile_keys(int cfg) { return kSegCfgs[cfg].waves * 64 * kSegCfgs[cfg].ipt; }

// Single-array sort of n <= kSmallSortMax keys in one launch (one workgroup, keys in registers and
// LDS): the smallest tile that holds them.  Up to 2048 keys 4 waves of 8 keys measured faster than
// 16 waves of 2 (10.2-11.4 against 11.8-12.0 us); from 2049 to 4096 keys 16 waves of 4 took 13.0
// against 16.0 us for the 8K-key tile.
template <int BITS, int WAVES, int IPT>
static void launch_small(hipStream_t s, const uint32_t* in, uint32_t* out, uint32_t n, uint32_t P, uint32_t* spl) {
  if (lane_order_ok())
    hipLaunchKernelGGL((k_sort_small<BITS, WAVES, IPT, seg_lcopies<BITS>(), SEG_RANK_ATOMIC>), dim3(1),
                       dim3(WAVES * 64), 0, s, in, out, n, P, spl);
  else
    hipLaunchKernelGGL((k_sort_small<BITS, WAVES, IPT, seg_lcopies<BITS>(), SEG_RANK_BALLOT>), dim3(1),
                       dim3(WAVES * 64), 0, s, in, out, n, P, spl);
}

ap_status enqueue_small_sort(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_spl,
                             hipStream_t s) {
  if (n > kSmallSortMax) return fail(AP_ERR_INVALID, "small sort takes at most %u keys", kSmallSortMax);
  const uint32_t nn = (uint32_t)n, PP = (uint32_t)P;
  uint32_t* spl = P > 1 ? d_spl : nullptr;
  prof_begin(AP_KIND_SEG, s);
  if (n <= 2048) launch_small<8, 4, 8>(s, d_in, d_out, nn, PP, spl);
  else if (n <= 4096) launch_small<8, 16, 4>(s, d_in, d_out, nn, PP, spl);
  else if (n <= 8192) launch_small<8, 16, 8>(s, d_in, d_out, nn, PP, spl);
  else launch_small<8, 16, 16>(s, d_in, d_out, nn, PP, spl);
  prof_end(s);
  return check_launch(s, "k_sort_small");
}

void seg_reset(hipStream_t s, SegCtl* ctl) { hipLaunchKernelGGL(k_seg_reset, dim3(1), dim3(64), 0, s, ctl); }

// Length groups: group g sorts the segments whose length class ceil(log2(length)) lies in
// [cls_lo, cls_hi] with kernel configuration cfg.  The defaults give each tile size its own
// classes: up to 2K keys with 2K-key tiles, (2K, 4K] with 4K-key tiles, (4K, 8K] with 8K-key
// tiles, and above 8K with 16K-key tiles (longer segments by digit sweeps).  Every group is one
// more concurrent persistent kernel, so classes sharing a configuration share a group.  The tuner
// rewrites the table (ap_segmented_set_group, ap_load_tuning).
static std::mutex g_grp_mu;
// length classes ceil(log2(len)): one group per tile size (16K keys, also taking longer segments; 8K; 4K; 2K)
static SegGroup g_groups[kSegGroups] = {{14, 31, 10}, {13, 13, 0}, {12, 12, 5}, {1, 11, 3}, {1, 0, 0}, {1, 0, 0}};
static int g_groups_version = 0;  // bumped on every change (invalidates captured graphs)

int seg_groups_version() {
  std::lock_guard<std::mutex> lk(g_grp_mu);
  return g_groups_version;
}

void seg_groups(SegGroup* out) {
  std::lock_guard<std::mutex> lk(g_grp_mu);
  for (int g = 0; g < kSegGroups; ++g) out[g] = g_groups[g];
}

// The used groups (cls_lo <= cls_hi) must cover every length class 1..31 exactly once.  Two
// groups sharing a class would both sort its segments, concurrently, in place through the same
// scratch; a class no group covers would never be sorted.  AP_ERR_INVALID otherwise.
ap_status seg_groups_check(const SegGroup* grp) {
  int owner[32];
  for (int c = 0; c < 32; ++c) owner[c] = -1;
  for (int g = 0; g < kSegGroups; ++g) {
    if (grp[g].cls_lo > grp[g].cls_hi) continue;
    if (grp[g].cls_lo < 1 || grp[g].cls_hi > 31)
      return fail(AP_ERR_INVALID, "length group %d: classes [%d, %d] outside [1, 31]", g, grp[g].cls_lo, grp[g].cls_hi);
    for (int c = grp[g].cls_lo; c <= grp[g].cls_hi; ++c) {
      if (owner[c] >= 0)
        return fail(AP_ERR_INVALID, "length groups %d and %d both cover length class %d", owner[c], g, c);
      owner[c] = g;
    }
  }
  for (int c = 1; c <= 31; ++c)
    if (owner[c] < 0) return fail(AP_ERR_INVALID, "no length group covers length class %d", c);
  return AP_OK;
}


// Segments of at least g_long_min keys (0 = none) are sorted by the device-wide passes over one
// flat tile space (apsort_seg_long.h); shorter ones by one workgroup each.
static std::atomic<size_t> g_long_min{(size_t)1 << 20};
constexpr uint32_t kLongTileMin = 16384;  // flat tile of the mask-rank shape; the atomic rank uses 32K

// Workspace: [SegCtl | pad to 256][order: nseg descriptors | pad][tmp n_total u32]
//            [long segments: descriptors | bucket counts 4x256 u32 | totals 4x256 u32]
//            [look-back words: 4 passes x flat tiles x 256 u32]
// Segments of long_min keys or more are disjoint, so at most n_total / long_min of them; their
// flat tiles number at most n_total / (16K-key tile) + one partial tile each.
struct SegLayout {
  size_t ctl, order, tmp, longs, lhist, lbase, lstatus, total;
  uint32_t nlong_max, tiles_max;
  size_t status_pass_words;
  uint32_t long_min;  // effective threshold (all-ones: no long path)
};
static size_t up256(size_t x) { return (x + 255) / 256 * 256; }
static SegLayout seg_layout(size_t n_total, int nseg, size_t long_min) {
  SegLayout L{};
  const bool longs = long_min >= 2 && long_min <= n_total;
  L.long_min = longs ? (uint32_t)long_min : 0xFFFFFFFFu;
  L.nlong_max = longs ? (uint32_t)(n_total / long_min) : 0u;
  L.tiles_max = longs ? (uint32_t)((n_total + kLongTileMin - 1) / kLongTileMin + L.nlong_max) : 0u;
  L.status_pass_words = (size_t)L.tiles_max * 256;
  size_t off = 0;
  L.ctl = off;     off += up256(sizeof(SegCtl));
  L.order = off;   off += up256(sizeof(SegDesc) * (size_t)std::max(nseg, 1));
  L.tmp = off;     off += up256(sizeof(uint32_t) * std::max<size_t>(n_total, 1));
  L.longs = off;   off += up256(sizeof(LongSeg) * L.nlong_max);
  L.lhist = off;   off += up256(sizeof(uint32_t) * 1024 * L.nlong_max);
  L.lbase = off;   off += up256(sizeof(uint32_t) * 1024 * L.nlong_max);
  L.lstatus = off; off += up256(sizeof(uint32_t) * 4 * L.status_pass_words);
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
  // length groups after the first, and the long segments' passes, run on streams of their own,
  // forked from and joined back to `stream` with events (created on first use)
  hipStream_t aux[kSegGroups + 1];
  hipEvent_t ev_fork;
  hipEvent_t ev_join[kSegGroups + 1];
};
static std::mutex g_seg_mu;
static std::vector<SegEntry> g_seg;

static ap_status seg_fork_objects(SegEntry& c) {
  if (c.ev_fork) return AP_OK;
  for (int g = 0; g <= kSegGroups; ++g) {
    hipError_t e = hipStreamCreateWithFlags(&c.aux[g], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.ev_join[g], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "segmented sort: auxiliary stream");
  }
  hipError_t e = hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming);
  return e == hipSuccess ? AP_OK : hip_fail(e, "segmented sort: fork event");
}

static ap_status seg_entry(hipStream_t s, size_t need, SegEntry** out, bool* fresh) {
  *fresh = false;
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
      // grow geometrically (at least by a quarter) so that slowly growing calls do not
      // reallocate every time
      const size_t bytes = std::max(need, c.bytes + c.bytes / 4);
      (void)hipFree(c.ws);
      c.ws = nullptr;
      c.bytes = 0;
      e = hipMalloc(&c.ws, bytes);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc(segmented workspace)");
      c.bytes = bytes;
      *fresh = true;
    }
    *out = &c;
    return seg_fork_objects(c);
  }
  SegEntry c{};
  c.dev = dev;
  c.stream = s;
  e = hipMalloc(&c.ws, need);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(segmented workspace)");
  c.bytes = need;
  g_seg.push_back(c);
  *out = &g_seg.back();
  *fresh = true;
  return seg_fork_objects(g_seg.back());
}

// A fresh workspace: zero the control block (offset 0 whatever the sizes; every call leaves it
// zero again).  Everything else is written by each call before it is read: the long segments'
// bucket counts, whose place depends on the call's sizes, are zeroed by k_seg_fill.
static ap_status seg_zero_fresh(void* ws, const SegLayout& L, hipStream_t s) {
  char* w = static_cast<char*>(ws);
  return fill_u32(reinterpret_cast<uint32_t*>(w + L.ctl), 0u, up256(sizeof(SegCtl)) / 4, s);
}

// The launch sequence: classify -> fill -> persistent sort.  No host synchronisation; every grid
// size is fixed by (nseg, device), so the sequence can be captured once and replayed.
ap_status enqueue_segmented(uint32_t* d_keys, size_t n_total, const uint32_t* d_off, int nseg, uint32_t* d_status,
                            void* ws, const SegLayout& L, int cfg, hipStream_t s, const hipStream_t* aux,
                            hipEvent_t ev_fork, const hipEvent_t* ev_join) {
  char* w = static_cast<char*>(ws);
  SegCtl* ctl = reinterpret_cast<SegCtl*>(w + L.ctl);
  SegDesc* order = reinterpret_cast<SegDesc*>(w + L.order);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(w + L.tmp);
  LongSeg* longs = reinterpret_cast<LongSeg*>(w + L.longs);
  uint32_t* lhist = reinterpret_cast<uint32_t*>(w + L.lhist);
  uint32_t* lbase = reinterpret_cast<uint32_t*>(w + L.lbase);
  uint32_t* lstatus = reinterpret_cast<uint32_t*>(w + L.lstatus);
  const int cus = device_cus();
  const bool atomic_rank = lane_order_ok();
  const uint32_t long_tile = atomic_rank ? 32768u : kLongTileMin;
  const uint32_t g1 = (uint32_t)std::min<int>((nseg + 255) / 256 + 1, 4 * cus);
  prof_begin(AP_KIND_SEG, s);
  hipLaunchKernelGGL(k_seg_classify, dim3(g1), dim3(256), 0, s, d_off, (uint32_t)nseg, (uint32_t)n_total,
                     L.long_min, ctl, d_status);
  hipLaunchKernelGGL(k_seg_fill, dim3(g1), dim3(256), 0, s, d_off, (uint32_t)nseg, (uint32_t)n_total, L.long_min,
                     long_tile, ctl, d_keys, tmp, order, longs, lhist);
  // One persistent kernel per length group.  The groups sort disjoint segments and take work from
  // counters of their own, so they run concurrently: the first group (longest segments) on `s`,
  // the others on auxiliary streams forked after k_seg_fill and joined before the reset.  A
  // group's workgroups then fill the CUs that another group's tail (its few longest segments)
  // leaves idle, instead of waiting for that kernel to end.
  SegGroup grp[kSegGroups];
  seg_groups(grp);
  hipError_t e = hipEventRecord(ev_fork, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord(fork)");
  bool first = true;
  for (int g = 0; g < kSegGroups; ++g) {
    if (grp[g].cls_lo > grp[g].cls_hi) continue;
    const dim3 grid(seg_workgroups(grp[g], (uint32_t)nseg));
    if (first) {
      launch_seg_group(grp[g], grid, s, order, 0u, ~0u, g, ctl);
      first = false;
      continue;
    }
    e = hipStreamWaitEvent(aux[g], ev_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(fork)");
    launch_seg_group(grp[g], grid, aux[g], order, 0u, ~0u, g, ctl);
    e = hipEventRecord(ev_join[g], aux[g]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev_join[g], 0);
    if (e != hipSuccess) return hip_fail(e, "segmented sort: join");
  }
  // Long segments: bucket counts, plans, four device-wide passes and the copy back, on a stream of
  // their own beside the group kernels.
  if (L.nlong_max) {
    hipStream_t ls = aux[kSegGroups];
    e = hipStreamWaitEvent(ls, ev_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(fork)");
    const uint32_t gp = std::min<uint32_t>(L.nlong_max, (uint32_t)(4 * cus));
    const uint32_t gc = std::min<uint32_t>(L.tiles_max, (uint32_t)(4 * cus));
    if (atomic_rank) {
      hipLaunchKernelGGL((k_seg_long_hist<32768>), dim3(cus), dim3(1024), 0, ls, ctl, longs, lhist, lstatus,
                         L.status_pass_words);
      hipLaunchKernelGGL(k_seg_long_plan, dim3(gp), dim3(256), 0, ls, ctl, longs, lhist, lbase);
      // plain stores before the last pass, the non-temporal hint on it (long segments hold at least
      // 2^20 keys each; the single-array sort does the same from 2^23 keys on)
      for (int d = 0; d < 3; ++d)
        hipLaunchKernelGGL((k_seg_long_pass<16, 32, RANK_ATOMIC, false>), dim3(cus), dim3(1024), 0, ls, ctl, longs,
                           lbase, lstatus + (size_t)d * L.status_pass_words, d);
      hipLaunchKernelGGL((k_seg_long_pass<16, 32, RANK_ATOMIC, true>), dim3(cus), dim3(1024), 0, ls, ctl, longs,
                         lbase, lstatus + (size_t)3 * L.status_pass_words, 3);
      hipLaunchKernelGGL((k_seg_long_copy<32768>), dim3(gc), dim3(256), 0, ls, ctl, longs);
    } else {
      hipLaunchKernelGGL((k_seg_long_hist<16384>), dim3(cus), dim3(1024), 0, ls, ctl, longs, lhist, lstatus,
                         L.status_pass_words);
      hipLaunchKernelGGL(k_seg_long_plan, dim3(gp), dim3(256), 0, ls, ctl, longs, lhist, lbase);
      for (int d = 0; d < 3; ++d)
        hipLaunchKernelGGL((k_seg_long_pass<8, 32, RANK_MATCH, false>), dim3(cus), dim3(512), 0, ls, ctl, longs,
                           lbase, lstatus + (size_t)d * L.status_pass_words, d);
      hipLaunchKernelGGL((k_seg_long_pass<8, 32, RANK_MATCH, true>), dim3(cus), dim3(512), 0, ls, ctl, longs, lbase,
                         lstatus + (size_t)3 * L.status_pass_words, 3);
      hipLaunchKernelGGL((k_seg_long_copy<16384>), dim3(gc), dim3(256), 0, ls, ctl, longs);
    }
    e = hipEventRecord(ev_join[kSegGroups], ls);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev_join[kSegGroups], 0);
    if (e != hipSuccess) return hip_fail(e, "segmented sort: join");
  }
  seg_reset(s, ctl);
  prof_end(s);
  (void)cfg;
  return check_launch(s, "k_seg_sort");
}

}  // namespace aps

using namespace aps;

extern "C" {

ap_status ap_sort_u32_segmented(uint32_t* d_keys, size_t n_total, const uint32_t* d_offsets, int nseg,
                                uint32_t* d_status, void* stream) {
  ApRange range("ap_sort_u32_segmented");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (nseg < 0) return fail(AP_ERR_INVALID, "nseg must be >= 0");
  if (n_total >= AP_MAX_KEYS) return fail(AP_ERR_INVALID, "n_total must be < 2^30");
  if (nseg == 0) return d_status ? fill_u32(d_status, 0u, 1, s) : AP_OK;
  if (!d_offsets) return fail(AP_ERR_INVALID, "d_offsets is NULL");
  if (n_total && !d_keys) return fail(AP_ERR_INVALID, "d_keys is NULL with n_total > 0");
  if (((uintptr_t)d_keys | (uintptr_t)d_offsets) & 3u) return fail(AP_ERR_INVALID, "pointers must be 4-byte aligned");
  {
    SegGroup grp[kSegGroups];
    seg_groups(grp);
    ap_status gst = seg_groups_check(grp);
    if (gst != AP_OK) return gst;
  }
  const SegLayout L = seg_layout(n_total, nseg, g_long_min.load());
  std::lock_guard<std::mutex> lk(g_seg_mu);
  SegEntry* ent = nullptr;
  bool fresh = false;
  ap_status st = seg_entry(s, L.total, &ent, &fresh);
  if (st != AP_OK) return st;
  if (fresh) {
    st = seg_zero_fresh(ent->ws, L, s);
    if (st != AP_OK) return st;
  }
  // graph key: the group table and the rank primitive (both baked into the captured kernels)
  const int cfg = seg_groups_version() * 2 + (lane_order_ok() ? 1 : 0);

  // Replay a captured graph when the call repeats the previous one on this stream; capture
  // otherwise (only on a non-default stream that is not itself being captured).
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (s) {
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  }
  const bool graphable = s != nullptr && cap == hipStreamCaptureStatusNone && !prof_active();
  if (!graphable) return enqueue_segmented(d_keys, n_total, d_offsets, nseg, d_status, ent->ws, L, cfg, s, ent->aux, ent->ev_fork,
                                              ent->ev_join);
  const bool same = ent->exec && ent->k_keys == d_keys && ent->k_n == n_total && ent->k_off == d_offsets &&
                    ent->k_nseg == nseg && ent->k_status == d_status && ent->k_cfg == cfg;
  if (!same) {
    if (ent->exec) {
      (void)hipGraphExecDestroy(ent->exec);
      ent->exec = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    st = enqueue_segmented(d_keys, n_total, d_offsets, nseg, d_status, ent->ws, L, cfg, s, ent->aux, ent->ev_fork,
                           ent->ev_join);
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
  return seg_layout(n_total, nseg, g_long_min.load()).total;
}

ap_status ap_segmented_set_long_min(size_t long_min) {
  if (long_min == 1) return fail(AP_ERR_INVALID, "long_min must be 0 (never) or at least 2");
  g_long_min.store(long_min);
  std::lock_guard<std::mutex> lk(g_grp_mu);
  ++g_groups_version;  // baked into captured graphs
  return AP_OK;
}

size_t ap_segmented_get_long_min(void) { return g_long_min.load(); }

ap_status ap_segmented_set_config(int cfg) {
  if (cfg < 0 || cfg >= kNumSegCfgs) return fail(AP_ERR_INVALID, "config index out of range");
  std::lock_guard<std::mutex> lk(g_grp_mu);
  for (auto& g : g_groups) g.cfg = cfg;
  ++g_groups_version;
  return AP_OK;
}

ap_status ap_segmented_set_group(int g, int cls_lo, int cls_hi, int cfg) {
  if (g < 0 || g >= kSegGroups) return fail(AP_ERR_INVALID, "group index out of range");
  if (cfg < 0 || cfg >= kNumSegCfgs) return fail(AP_ERR_INVALID, "config index out of range");
  if (cls_lo < 1 || cls_hi > 31) return fail(AP_ERR_INVALID, "length classes must lie in [1, 31]");
  std::lock_guard<std::mutex> lk(g_grp_mu);
  g_groups[g] = SegGroup{cls_lo, cls_hi, cfg};
  ++g_groups_version;
  return AP_OK;
}

ap_status ap_segmented_get_group(int g, int* cls_lo, int* cls_hi, int* cfg) {
  if (g < 0 || g >= kSegGroups || !cls_lo || !cls_hi || !cfg) return fail(AP_ERR_INVALID, "bad argument");
  std::lock_guard<std::mutex> lk(g_grp_mu);
  *cls_lo = g_groups[g].cls_lo;
  *cls_hi = g_groups[g].cls_hi;
  *cfg = g_groups[g].cfg;
  return AP_OK;
}

ap_status ap_load_tuning(const char* path) {
  if (!path) return fail(AP_ERR_INVALID, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(AP_ERR_INVALID, "cannot open tuning table %s", path);
  SegGroup next[kSegGroups];
  for (auto& g : next) g = SegGroup{1, 0, 0};
  char line[256];
  int seen = 0;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    int g, lo, hi, c;
    if (std::sscanf(line, "%d %d %d %d", &g, &lo, &hi, &c) != 4) continue;
    if (g < 0 || g >= kSegGroups || c < 0 || c >= kNumSegCfgs || lo < 1 || hi > 31) {
      std::fclose(f);
      return fail(AP_ERR_INVALID, "bad tuning line: %s", line);
    }
    next[g] = SegGroup{lo, hi, c};
    ++seen;
  }
  std::fclose(f);
  if (!seen) return fail(AP_ERR_INVALID, "no tuning entries in %s", path);
  ap_status st = seg_groups_check(next);
  if (st != AP_OK) return st;
  std::lock_guard<std::mutex> lk(g_grp_mu);
  for (int g = 0; g < kSegGroups; ++g) g_groups[g] = next[g];
  ++g_groups_version;
  return AP_OK;
}

int ap_segmented_num_configs(void) { return kNumSegCfgs; }

int ap_segmented_num_groups(void) { return kSegGroups; }

ap_status ap_segmented_config_info(int cfg, int* digit_bits, int* waves, int* keys_per_lane) {
  if (cfg < 0 || cfg >= kNumSegCfgs || !digit_bits || !waves || !keys_per_lane)
    return fail(AP_ERR_INVALID, "bad argument");
  *digit_bits = kSegCfgs[cfg].bits;
  *waves = kSegCfgs[cfg].waves;
  *keys_per_lane = kSegCfgs[cfg].ipt;
  return AP_OK;
}

}  // extern "C"
