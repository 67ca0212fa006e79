// Host side of libapsort.so: argument checks, workspace layout and cache, launch sequence, and the
// C entry points declared in include/apsort.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "apsort.h"
#include "apsort_kernels.h"
#include "apsort_internal.h"

namespace aps {

// ---------------------------------------------------------------- errors
static thread_local std::string t_err;

ap_status fail(ap_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return st;
}

ap_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? AP_ERR_NOMEM : AP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static bool debug_sync() {
  static const bool on = [] {
    const char* s = std::getenv("AP_DEBUG_SYNC");
    return s && s[0] && s[0] != '0';
  }();
  return on;
}

ap_status check_launch(hipStream_t s, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  if (debug_sync()) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, what);
  }
  return AP_OK;
}

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  static std::mutex mu;
  static std::vector<int> cus;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cus.size() <= dev) cus.resize(dev + 1, 0);
  if (!cus[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cus[dev] = v;
  }
  return cus[dev];
}

// ---------------------------------------------------------------- lane-order check
// The atomic rank of k_pass needs the LDS to service the conflicting lanes of one atomic
// instruction in lane order.  k_lane_order_probe checks that once per device; until a device has
// passed the check, or if it fails, the passes use the order-agnostic match rank.
static std::mutex g_lane_mu;
static std::vector<int> g_lane_state;  // per device: -1 unknown, 0 failed, 1 passed

static int g_force_match = 0;  // testing hook: 1 = always use the match rank

bool lane_order_ok() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_lane_mu);
  return !g_force_match && dev < (int)g_lane_state.size() && g_lane_state[dev] == 1;
}

int lane_order_state() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::lock_guard<std::mutex> lk(g_lane_mu);
  return dev < (int)g_lane_state.size() ? g_lane_state[dev] : -1;
}

void set_rank_mode(int mode) {
  std::lock_guard<std::mutex> lk(g_lane_mu);
  g_force_match = mode == 1 ? 1 : 0;
}

ap_status check_lane_order(hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  {
    std::lock_guard<std::mutex> lk(g_lane_mu);
    if ((int)g_lane_state.size() <= dev) g_lane_state.resize(dev + 1, -1);
    if (g_lane_state[dev] != -1) return AP_OK;
  }
  uint32_t* d_flag = nullptr;
  e = hipMalloc(&d_flag, 256);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(lane-order flag)");
  uint32_t h_flag = 1u;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, d_flag, 0u, (size_t)1);
  hipLaunchKernelGGL(k_lane_order_probe, dim3(64), dim3(256), 0, s, d_flag, 180u);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&h_flag, d_flag, sizeof h_flag, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_flag);
  if (e != hipSuccess) return hip_fail(e, "lane-order check");
  std::lock_guard<std::mutex> lk(g_lane_mu);
  g_lane_state[dev] = (h_flag == 0u) ? 1 : 0;
  return AP_OK;
}

// ---------------------------------------------------------------- configuration
// Digit width and tile shapes of the single-array sort.  8-bit digits (4 passes for 32-bit keys).
// Every tile is one workgroup of 16 waves; the tile grows with n (4, 8, 16 then 32 keys per
// lane).  Larger tiles mean fewer tiles, so the look-back chain between tiles is shorter relative
// to the time between tile starts, and a bucket's run in a tile is longer, so the scatter writes
// longer contiguous pieces.  The largest tile (32 keys per lane, 148 KiB of LDS, one workgroup per
// CU) is used from 2^22 keys on, although below 2^23 keys its 128-255 tiles leave CUs idle: a
// tile's phases are latency-bound, and fewer, larger tiles finish a pass sooner.  Sixteen waves
// split a tile's serial work (load, rank, reorder, scatter: one step per key of a lane) into
// fewer steps than 4 or 8 waves holding the same tile.  Shapes and thresholds are the fastest by
// measured sort time at every power of two and 1.5 times one from 2^15 to 1.5 * 2^25 keys.
constexpr int kBits = 8;
constexpr int kRadix = 1 << kBits;
constexpr int kDigits = (32 + kBits - 1) / kBits;
constexpr int kHistThreads = 1024;  // one workgroup per CU (grid <= CUs)
constexpr uint32_t kHistCopies = kHistMaxCopies;  // copies of the global counters (contention / 32)

struct PassShape {
  int waves, ipt;
};
static const PassShape kShapes[] = {{16, 4}, {16, 8}, {16, 16}, {16, 32}};  // 4K, 8K, 16K, 32K keys

static int shape_for(size_t n) {
  if (n >= ((size_t)1 << 22)) return 3;
  if (n >= ((size_t)1 << 20)) return 2;
  if (n >= ((size_t)1 << 17)) return 1;
  return 0;
}
// The mask rank needs extra LDS that the 32K-key tile cannot spare; it uses the 16K-key shape.
static int shape_for_rank(size_t n, bool atomic_rank) {
  const int sh = shape_for(n);
  return (!atomic_rank && sh == 3) ? 2 : sh;
}
static int tile_keys(int sh) { return kShapes[sh].waves * 64 * kShapes[sh].ipt; }

// Tile shape override (ap_set_pass_shape): -1 = by size.
static std::atomic<int> g_shape_override{-1};
static int shape_used(size_t n, bool atomic_rank) {
  const int o = g_shape_override.load();
  if (o >= 0) return (!atomic_rank && o == 3) ? 2 : o;
  return shape_for_rank(n, atomic_rank);
}

// LDS copies of the counters in k_hist_plan: as many as fit in 64 KiB, at most 16.
template <int BITS>
constexpr int hist_lcopies() {
  constexpr int hw = ((32 + BITS - 1) / BITS) << BITS;
  constexpr int c = 16384 / (hw + 1);
  return c < 1 ? 1 : (c > 16 ? 16 : c);
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workgroups of k_hist_plan: 16 keys per thread or more, at most one workgroup per CU, but never
// so few that a thread counts more than kHistMaxVecPerThread vectors of 4 keys (the 16-bit lane
// copies of the counters would overflow).
static uint32_t hist_grid(size_t n, int cus) {
  size_t g = std::min<size_t>((n + (size_t)kHistThreads * 16 - 1) / ((size_t)kHistThreads * 16), (size_t)cus);
  const size_t per_wg_max = (size_t)kHistThreads * 4 * kHistMaxVecPerThread;
  g = std::max<size_t>(g, (n + per_wg_max - 1) / per_wg_max);
  return (uint32_t)std::max<size_t>(g, 1);
}

// Pairs (key + value) stage the values beside the keys in LDS, so their tile is at most 16K keys
// (16 waves x 16 keys with the atomic rank; 8 x 32 with the mask rank, whose words would not fit
// beside both stages with 16 waves), and below 2^22 pairs the 8K-key tile measured faster than
// the 16K one.
static int shape_for_pairs(size_t n) {
  const int sh = shape_used(n, true);
  if (g_shape_override.load() >= 0) return std::min(sh, 2);
  return std::min(sh, n >= ((size_t)1 << 22) ? 2 : 1);
}

// Workspace layout (bytes from the 256-byte aligned base):
//   [hist copies*D*R u32][base D*R u32][plan 32 u32][done 1 u32 | pad][tile counters 8 u32 | pad]
//   [status D * ntiles * R u32][tmp n u32][pairs only: value tmp n u32]
// hist and done are self-clearing; tile counters and the used part of status are cleared by
// k_hist_plan.  Status capacity covers the smaller tile of either rank primitive.
Layout layout_for(size_t n, bool pairs) {
  Layout L{};
  const int T = pairs ? tile_keys(std::min(shape_for_pairs(n), shape_used(n, false)))
                      : std::min(tile_keys(shape_used(n, true)), tile_keys(shape_used(n, false)));
  L.tile_keys = T;
  L.ntiles = (uint32_t)((n + T - 1) / T);
  size_t off = 0;
  L.hist = off;   off += align_up(sizeof(uint32_t) * kHistCopies * kDigits * kRadix, 256);
  L.base = off;   off += align_up(sizeof(uint32_t) * kDigits * kRadix, 256);
  L.plan = off;   off += align_up(sizeof(uint32_t) * PL_WORDS, 256);
  L.done = off;   off += 256;
  L.tctr = off;   off += 256;
  L.status = off; off += align_up(sizeof(uint32_t) * (size_t)kDigits * L.ntiles * kRadix, 256);
  L.zero_bytes = off - L.tctr;  // upper bound of the region k_hist_plan clears
  L.tmp = off;    off += align_up(sizeof(uint32_t) * n, 256);
  L.vtmp = off;
  if (pairs) off += align_up(sizeof(uint32_t) * n, 256);
  L.total = off;
  L.init_bytes = L.tctr;        // hist, base, plan, done: zeroed once at workspace creation
  return L;
}

// Store hint of the keys-only scatter, by array size and pass.  From 2^23 keys on, the passes
// before the last store plainly: the next pass finds much of its input still in the 256 MB
// last-level cache, and run-boundary lines shared by two tiles merge there instead of reaching
// HBM twice as partial lines.  The last pass keeps the non-temporal hint, so that a sort pays the
// write-back of its own output instead of leaving dirty lines to the next kernel.  Measured per
// sort of uniform keys against the hint on every pass: 0.593 vs 0.623 ms at 2^26, 2.357 vs 2.477
// at 2^28, 0.894 vs 0.978 at 3*2^25; below 2^23 plain stores are slower (2^22: 0.092 vs 0.087).
static bool keys_store_nt(size_t n, int d) { return n < ((size_t)1 << 23) || d == kDigits - 1; }

// Load hint of the pairs pass by array size.  Measured per pairs sort of uniform keys: loads with
// the non-temporal hint are 6-11% faster from 2^24 to 2^25 pairs and 3-4% up to 5*2^23 (128-320
// MiB of keys and values, where the dead input lines then leave the last-level cache to the
// output the next pass reads), no faster at 2^22-3*2^22, and 1% slower at 3*2^24 and 2^26.
static bool pairs_load_nt(size_t n) { return n >= ((size_t)1 << 24) && n <= ((size_t)5 << 23); }

template <int W, int I, bool KV, bool MATCH, bool NT, bool NTL = false>
static void launch_pass_hint(bool atomic_rank, dim3 grid, hipStream_t s, const uint32_t* in, uint32_t* out,
                             uint32_t* tmp, uint32_t n, int d, const uint32_t* plan, const uint32_t* base_d,
                             uint32_t* st_d, uint32_t* tctr, const uint32_t* vin, uint32_t* vout, uint32_t* vtmp) {
  if constexpr (MATCH && W * 64 * I <= 16384) {
    if (!atomic_rank) {
      hipLaunchKernelGGL((k_pass<kBits, W, I, RANK_MATCH, 4, KV, NT, NTL>), grid, dim3(W * 64), 0, s, in, out, tmp,
                         n, d, plan, base_d, st_d, tctr, vin, vout, vtmp);
      return;
    }
  }
  hipLaunchKernelGGL((k_pass<kBits, W, I, RANK_ATOMIC, 4, KV, NT, NTL>), grid, dim3(W * 64), 0, s, in, out, tmp, n,
                     d, plan, base_d, st_d, tctr, vin, vout, vtmp);
}

// MATCH = false builds only the atomic-rank kernel (for shapes whose mask-rank words would not fit
// the LDS); the caller then passes atomic_rank = true.  The size-dependent hints (plain stores for
// keys, non-temporal loads for pairs) are built only for the tiles of 16K keys and more, the
// shapes chosen at the sizes where they pay; a smaller tile forced at those sizes keeps the
// default accesses.
template <int W, int I, bool KV, bool MATCH = true>
static void launch_pass(bool atomic_rank, dim3 grid, hipStream_t s, const uint32_t* in, uint32_t* out, uint32_t* tmp,
                        uint32_t n, int d, const uint32_t* plan, const uint32_t* base_d, uint32_t* st_d,
                        uint32_t* tctr, const uint32_t* vin, uint32_t* vout, uint32_t* vtmp) {
  if constexpr (!KV && W * 64 * I >= 16384) {
    if (!keys_store_nt(n, d)) {
      launch_pass_hint<W, I, KV, MATCH, false>(atomic_rank, grid, s, in, out, tmp, n, d, plan, base_d, st_d, tctr,
                                               vin, vout, vtmp);
      return;
    }
  }
  if constexpr (KV && W * 64 * I >= 16384) {
    if (pairs_load_nt(n)) {
      launch_pass_hint<W, I, KV, MATCH, true, true>(atomic_rank, grid, s, in, out, tmp, n, d, plan, base_d, st_d,
                                                    tctr, vin, vout, vtmp);
      return;
    }
  }
  launch_pass_hint<W, I, KV, MATCH, true>(atomic_rank, grid, s, in, out, tmp, n, d, plan, base_d, st_d, tctr, vin,
                                          vout, vtmp);
}

// Debug mode of the digit pass (ap_debug_pass): the keys-only passes then run k_pass_dbg.
struct PassDebugState {
  int mode;
  uint64_t seed;
  unsigned long long* trace;
  uint64_t trace_records;
};
static std::mutex g_dbg_mu;
static PassDebugState g_dbg{PASS_DBG_NONE, 0, nullptr, 0};
static PassDebugState pass_debug() {
  std::lock_guard<std::mutex> lk(g_dbg_mu);
  return g_dbg;
}

template <int W, int I, int DBG>
static void launch_pass_dbg_mode(bool atomic_rank, dim3 grid, hipStream_t s, const uint32_t* in, uint32_t* out,
                                 uint32_t* tmp, uint32_t n, int d, const uint32_t* plan, const uint32_t* base_d,
                                 uint32_t* st_d, uint32_t* tctr, const PassDebugArgs& a) {
  if constexpr (W * 64 * I <= 16384) {
    if (!atomic_rank) {
      hipLaunchKernelGGL((k_pass_dbg<kBits, W, I, RANK_MATCH, DBG>), grid, dim3(W * 64), 0, s, in, out, tmp, n, d,
                         plan, base_d, st_d, tctr, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_pass_dbg<kBits, W, I, RANK_ATOMIC, DBG>), grid, dim3(W * 64), 0, s, in, out, tmp, n, d, plan,
                     base_d, st_d, tctr, a);
}
template <int W, int I>
static void launch_pass_dbg(const PassDebugState& st, bool atomic_rank, dim3 grid, hipStream_t s, const uint32_t* in,
                            uint32_t* out, uint32_t* tmp, uint32_t n, int d, uint32_t ntiles, const uint32_t* plan,
                            const uint32_t* base_d, uint32_t* st_d, uint32_t* tctr) {
  PassDebugArgs a{};
  a.seed = st.seed;
  a.trace = st.trace;
  a.trace_records = st.trace_records;
  a.record0 = (uint32_t)d * ntiles;
  if (st.mode == PASS_DBG_PERTURB)
    launch_pass_dbg_mode<W, I, PASS_DBG_PERTURB>(atomic_rank, grid, s, in, out, tmp, n, d, plan, base_d, st_d, tctr, a);
  else
    launch_pass_dbg_mode<W, I, PASS_DBG_TRACE>(atomic_rank, grid, s, in, out, tmp, n, d, plan, base_d, st_d, tctr, a);
}

// ---------------------------------------------------------------- launch sequence
ap_status enqueue_sort(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_spl,
                       void* ws, const Layout& L, hipStream_t s, const uint32_t* d_vin, uint32_t* d_vout,
                       int first_digit) {
  return enqueue_sort_parts(d_in, d_out, n, P, d_spl, ws, static_cast<char*>(ws) + L.tctr, L, s, d_vin, d_vout,
                            first_digit);
}

ap_status enqueue_sort_parts(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_spl, void* ctl,
                             void* scratch, const Layout& L, hipStream_t s, const uint32_t* d_vin, uint32_t* d_vout,
                             int first_digit) {
  char* c = static_cast<char*>(ctl);
  char* w = static_cast<char*>(scratch);  // holds the layout from L.tctr on
  uint32_t* hist = reinterpret_cast<uint32_t*>(c + L.hist);
  uint32_t* base = reinterpret_cast<uint32_t*>(c + L.base);
  uint32_t* plan = reinterpret_cast<uint32_t*>(c + L.plan);
  uint32_t* done = reinterpret_cast<uint32_t*>(c + L.done);
  uint32_t* tctr = reinterpret_cast<uint32_t*>(w);
  uint32_t* status = reinterpret_cast<uint32_t*>(w + (L.status - L.tctr));
  uint32_t* tmp = reinterpret_cast<uint32_t*>(w + (L.tmp - L.tctr));
  const bool pairs = d_vout != nullptr;
  uint32_t* vtmp = pairs ? reinterpret_cast<uint32_t*>(w + (L.vtmp - L.tctr)) : nullptr;
  const uint32_t nn = (uint32_t)n;
  const int cus = device_cus();
  const int inplace = (d_in == d_out) ? 1 : 0;
  const bool atomic_rank = lane_order_ok();
  const int sh = pairs ? std::min(shape_for_pairs(n), shape_used(n, atomic_rank)) : shape_used(n, atomic_rank);
  const int T = tile_keys(sh);
  const uint32_t ntiles = (uint32_t)((n + T - 1) / T);
  if (ntiles > L.ntiles) return fail(AP_ERR_INVALID, "workspace sized for a larger tile (shape changed after sizing)");
  const size_t zero_bytes = 256 + align_up(sizeof(uint32_t) * (size_t)kDigits * ntiles * kRadix, 256);

  // A1 + A2
  {
    const uint32_t g = hist_grid(n, cus);
    prof_begin(AP_KIND_HIST, s);
    hipLaunchKernelGGL((k_hist_plan<kBits, kHistThreads, hist_lcopies<kBits>()>), dim3(g), dim3(kHistThreads), 0, s,
                       d_in, nn,
                       hist, base, plan, done, reinterpret_cast<uint4*>(tctr), (uint32_t)(zero_bytes / 16),
                       inplace, (uint32_t*)nullptr, kHistCopies, first_digit);
    prof_end(s);
    ap_status st = check_launch(s, "k_hist_plan");
    if (st != AP_OK) return st;
  }
  // A3-A6: one launch per digit; passes the plan skips exit at once
  const PassDebugState dbg = pass_debug();
  for (int d = 0; d < kDigits; ++d) {
    uint32_t* st_d = status + (size_t)d * ntiles * kRadix;
    const uint32_t* base_d = base + d * kRadix;
    prof_begin(AP_KIND_PASS + d, s);
    const dim3 grid(ntiles);
#define APS_PASS(W, I, KV)                                                                                      \
  if (!KV && dbg.mode != PASS_DBG_NONE)                                                                          \
    launch_pass_dbg<W, I>(dbg, atomic_rank, grid, s, d_in, d_out, tmp, nn, d, ntiles, plan, base_d, st_d, tctr); \
  else                                                                                                           \
    launch_pass<W, I, KV>(atomic_rank, grid, s, d_in, d_out, tmp, nn, d, plan, base_d, st_d, tctr, d_vin, d_vout, vtmp)
    if (pairs) {
      switch (sh) {
        case 2:
          // 16 waves when the atomic rank runs; the mask rank's words fit beside both stages only
          // with 8 waves (same 16K-key tile)
          if (atomic_rank)
            launch_pass<16, 16, true, false>(true, grid, s, d_in, d_out, tmp, nn, d, plan, base_d, st_d, tctr, d_vin,
                                             d_vout, vtmp);
          else
            APS_PASS(8, 32, true);
          break;
        case 1: APS_PASS(16, 8, true); break;
        default: APS_PASS(16, 4, true); break;
      }
    } else {
      switch (sh) {
        case 3: APS_PASS(16, 32, false); break;
        case 2: APS_PASS(16, 16, false); break;
        case 1: APS_PASS(16, 8, false); break;
        default: APS_PASS(16, 4, false); break;
      }
    }
#undef APS_PASS
    prof_end(s);
    ap_status st = check_launch(s, "k_pass");
    if (st != AP_OK) return st;
  }
  // A7
  {
    const size_t work = std::max<size_t>((pairs ? n / 2 : n / 4), (size_t)P);
    uint32_t g = (uint32_t)std::min<size_t>((work + 255 * 8) / (256 * 8), (size_t)4 * cus);
    g = std::max<uint32_t>(g, 1);
    prof_begin(AP_KIND_FINAL, s);
    hipLaunchKernelGGL(k_finalize, dim3(g), dim3(256), 0, s, d_in, d_out, tmp, nn, plan, (uint32_t)P,
                       P > 1 ? d_spl : nullptr, d_vin, d_vout, vtmp);
    prof_end(s);
    ap_status st = check_launch(s, "k_finalize");
    if (st != AP_OK) return st;
  }
  return AP_OK;
}

ap_status enqueue_finalize(const uint32_t* d_in, uint32_t* d_out, const uint32_t* tmp, size_t n, const uint32_t* plan,
                           int P, uint32_t* d_spl, hipStream_t s) {
  const size_t work = std::max<size_t>(n / 4, (size_t)P);
  uint32_t g = (uint32_t)std::min<size_t>((work + 255 * 8) / (256 * 8), (size_t)4 * device_cus());
  g = std::max<uint32_t>(g, 1);
  prof_begin(AP_KIND_FINAL, s);
  hipLaunchKernelGGL(k_finalize, dim3(g), dim3(256), 0, s, d_in, d_out, tmp, (uint32_t)n, plan, (uint32_t)P,
                     P > 1 ? d_spl : nullptr, (const uint32_t*)nullptr, (uint32_t*)nullptr, (const uint32_t*)nullptr);
  prof_end(s);
  return check_launch(s, "k_finalize");
}

ap_status fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s) {
  if (!count) return AP_OK;
  uint32_t g = (uint32_t)std::min<size_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, s, p, value, count);
  return check_launch(s, "k_fill_u32");
}

// Inspection entry point: k_hist_plan alone with a given digit width, on a small per-device
// control block (4 copies of up to 8192 counters, base, plan, done) that stays zero between calls.
template <int BITS>
static ap_status launch_plan_only(const uint32_t* d_in, uint32_t n, uint32_t* ctl, uint32_t* d_hist,
                                  uint32_t* d_plan, hipStream_t s) {
  constexpr int R = 1 << BITS, D = (32 + BITS - 1) / BITS;
  uint32_t* hist = ctl;                          // 4 x 8192 words
  uint32_t* base = ctl + 4 * 8192;               // 8192 words
  uint32_t* plan = ctl + 5 * 8192;               // PL_WORDS
  uint32_t* done = ctl + 5 * 8192 + PL_WORDS;
  const int cus = device_cus();
  const uint32_t g = hist_grid(n, cus);
  hipLaunchKernelGGL((k_hist_plan<BITS, kHistThreads, hist_lcopies<BITS>()>), dim3(g), dim3(kHistThreads), 0, s,
                     d_in, n, hist, base,
                     plan, done, (uint4*)nullptr, 0u, 0, d_hist, 4u, 0);
  ap_status st = check_launch(s, "k_hist_plan");
  if (st != AP_OK || !d_plan) return st;
  // d_plan[d] = run flag of pass d, d_plan[D] = number of passes
  hipError_t e = hipMemcpyAsync(d_plan, plan + PL_RUN, sizeof(uint32_t) * D, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_plan + D, plan + PL_NPASS, sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
  (void)R;
  return e == hipSuccess ? AP_OK : hip_fail(e, "hipMemcpyAsync(plan)");
}

ap_status enqueue_digit_plan(const uint32_t* d_in, size_t n, int bits, uint32_t* d_hist, uint32_t* d_plan,
                             hipStream_t s) {
  static std::mutex mu;
  static std::vector<uint32_t*> ctl_per_dev;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  uint32_t* ctl = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    if ((int)ctl_per_dev.size() <= dev) ctl_per_dev.resize(dev + 1, nullptr);
    if (!ctl_per_dev[dev]) {
      uint32_t* p = nullptr;
      e = hipMalloc(&p, sizeof(uint32_t) * (5 * 8192 + 256));
      if (e != hipSuccess) return hip_fail(e, "hipMalloc(plan control block)");
      ap_status st = fill_u32(p, 0u, 5 * 8192 + 256, s);
      if (st != AP_OK) return st;
      ctl_per_dev[dev] = p;
    }
    ctl = ctl_per_dev[dev];
  }
  const int D = (32 + bits - 1) / bits;
  if (n == 0) {
    ap_status st = fill_u32(d_hist, 0u, (size_t)D << bits, s);
    if (st == AP_OK && d_plan) st = fill_u32(d_plan, 0u, (size_t)D + 1, s);
    return st;
  }
  const uint32_t nn = (uint32_t)n;
  switch (bits) {
    case 4: return launch_plan_only<4>(d_in, nn, ctl, d_hist, d_plan, s);
    case 5: return launch_plan_only<5>(d_in, nn, ctl, d_hist, d_plan, s);
    case 6: return launch_plan_only<6>(d_in, nn, ctl, d_hist, d_plan, s);
    case 7: return launch_plan_only<7>(d_in, nn, ctl, d_hist, d_plan, s);
    case 8: return launch_plan_only<8>(d_in, nn, ctl, d_hist, d_plan, s);
    case 9: return launch_plan_only<9>(d_in, nn, ctl, d_hist, d_plan, s);
    case 10: return launch_plan_only<10>(d_in, nn, ctl, d_hist, d_plan, s);
    case 11: return launch_plan_only<11>(d_in, nn, ctl, d_hist, d_plan, s);
    default: return fail(AP_ERR_INVALID, "digit_bits must be in [4, 11]");
  }
}

ap_status check_sort_args(const uint32_t* d_in, const uint32_t* d_out, size_t n, int P) {
  if (P < 1) return fail(AP_ERR_INVALID, "P must be >= 1 (got %d)", P);
  if (n >= AP_MAX_KEYS) return fail(AP_ERR_INVALID, "n must be < 2^30 (got %zu)", n);
  if (n == 0) return AP_OK;
  if (!d_in || !d_out) return fail(AP_ERR_INVALID, "NULL key buffer with n > 0");
  if (((uintptr_t)d_in | (uintptr_t)d_out) & 3u) return fail(AP_ERR_INVALID, "key buffers must be 4-byte aligned");
  if (d_in != d_out) {
    const uintptr_t a0 = (uintptr_t)d_in, a1 = a0 + n * 4, b0 = (uintptr_t)d_out, b1 = b0 + n * 4;
    if (a0 < b1 && b0 < a1) return fail(AP_ERR_INVALID, "input and output overlap without being equal");
  }
  return AP_OK;
}

// Pairs: the keys' rules for the values, both arrays in place or neither, and no key array
// overlapping a value array.
static ap_status check_pairs_args(const uint32_t* kin, const uint32_t* vin, const uint32_t* kout,
                                  const uint32_t* vout, size_t n, int P) {
  ap_status st = check_sort_args(kin, kout, n, P);
  if (st == AP_OK) st = check_sort_args(vin, vout, n, P);
  if (st != AP_OK || n == 0) return st;
  if ((kin == kout) != (vin == vout))
    return fail(AP_ERR_INVALID, "keys and values must both be sorted in place or both out of place");
  const uintptr_t ks[2] = {(uintptr_t)kin, (uintptr_t)kout}, vs[2] = {(uintptr_t)vin, (uintptr_t)vout};
  for (uintptr_t a : ks)
    for (uintptr_t b : vs)
      if (a < b + n * 4 && b < a + n * 4) return fail(AP_ERR_INVALID, "a key array overlaps a value array");
  return AP_OK;
}

static ap_status pairs_with_ws(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, size_t n,
                               int P, uint32_t* d_spl, void* ws, size_t ws_bytes, hipStream_t s) {
  if (n == 0) return P > 1 && d_spl ? fill_u32(d_spl, 0xFFFFFFFFu, (size_t)P - 1, s) : AP_OK;
  const Layout L = layout_for(n, true);
  if (!ws || ws_bytes < L.total) return fail(AP_ERR_INVALID, "workspace too small: %zu < %zu", ws_bytes, L.total);
  if ((uintptr_t)ws & 255u) return fail(AP_ERR_INVALID, "workspace must be 256-byte aligned");
  return enqueue_sort(kin, kout, n, P, d_spl, ws, L, s, vin, vout);
}

ap_status sort_with_ws(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_spl, void* ws,
                       size_t ws_bytes, hipStream_t s) {
  if (n == 0) return P > 1 && d_spl ? fill_u32(d_spl, 0xFFFFFFFFu, (size_t)P - 1, s) : AP_OK;
  const Layout L = layout_for(n);
  if (!ws || ws_bytes < L.total) return fail(AP_ERR_INVALID, "workspace too small: %zu < %zu", ws_bytes, L.total);
  if ((uintptr_t)ws & 255u) return fail(AP_ERR_INVALID, "workspace must be 256-byte aligned");
  return enqueue_sort(d_in, d_out, n, P, d_spl, ws, L, s);
}

// ---------------------------------------------------------------- workspace cache
struct CacheEntry {
  int dev;
  hipStream_t stream;
  void* ptr;
  size_t bytes;
};
static std::mutex g_cache_mu;
static std::vector<CacheEntry> g_cache;

ap_status cached_workspace(size_t need, hipStream_t s, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  ap_status cst = check_lane_order(s);
  if (cst != AP_OK) return cst;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& c : g_cache) {
    if (c.dev == dev && c.stream == s) {
      if (c.bytes >= need) {
        *out = c.ptr;
        return AP_OK;
      }
      e = hipStreamSynchronize(s);  // the old block may still be in use on this stream
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      // grow geometrically (at least by a quarter) so that slowly growing calls do not
      // reallocate every time
      const size_t bytes = std::max(need, c.bytes + c.bytes / 4);
      (void)hipFree(c.ptr);
      c.ptr = nullptr;
      c.bytes = 0;
      e = hipMalloc(&c.ptr, bytes);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
      c.bytes = bytes;
      ap_status st = fill_u32(static_cast<uint32_t*>(c.ptr), 0u, layout_for(0).init_bytes / 4, s);
      if (st != AP_OK) return st;
      *out = c.ptr;
      return AP_OK;
    }
  }
  CacheEntry c{dev, s, nullptr, need};
  e = hipMalloc(&c.ptr, need);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
  ap_status st = fill_u32(static_cast<uint32_t*>(c.ptr), 0u, layout_for(0).init_bytes / 4, s);
  if (st != AP_OK) {
    (void)hipFree(c.ptr);
    return st;
  }
  g_cache.push_back(c);
  *out = c.ptr;
  return AP_OK;
}

ap_status release_cache() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  std::vector<CacheEntry> keep;
  for (auto& c : g_cache) {
    if (c.dev == dev) (void)hipFree(c.ptr);
    else keep.push_back(c);
  }
  g_cache.swap(keep);
  release_merge_scratch(dev);
  return AP_OK;
}

}  // namespace aps

// ================================================================ C ABI
using namespace aps;

extern "C" {

const char* ap_last_error(void) { return t_err.c_str(); }

const char* ap_version(void) { return "apsort 0.1 gfx950"; }

size_t ap_sort_workspace_bytes(size_t n) {
  if (n >= AP_MAX_KEYS) return 0;
  return layout_for(n).total;
}

ap_status ap_workspace_init(void* d_ws, size_t ws_bytes, void* stream) {
  const size_t need = layout_for(0).init_bytes;
  if (!d_ws || ws_bytes < need) return fail(AP_ERR_INVALID, "workspace too small for its control block");
  if ((uintptr_t)d_ws & 255u) return fail(AP_ERR_INVALID, "workspace must be 256-byte aligned");
  ap_status st = check_lane_order(static_cast<hipStream_t>(stream));
  if (st != AP_OK) return st;
  return fill_u32(static_cast<uint32_t*>(d_ws), 0u, need / 4, static_cast<hipStream_t>(stream));
}

ap_status ap_sort_u32(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_splitters,
                      void* stream) {
  ApRange range("ap_sort_u32");
  ap_status st = check_sort_args(d_in, d_out, n, P);
  if (st != AP_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) return sort_with_ws(d_in, d_out, 0, P, d_splitters, nullptr, 0, s);
  // A short array is sorted in one launch by one workgroup (unless a pass shape is forced, which
  // pins the device-wide kernels at every size).
  if (n <= kSmallSortMax && g_shape_override.load() < 0) {
    st = check_lane_order(s);
    if (st != AP_OK) return st;
    return enqueue_small_sort(d_in, d_out, n, P, d_splitters, s);
  }
  const Layout L = layout_for(n);
  void* ws = nullptr;
  st = cached_workspace(L.total, s, &ws);
  if (st != AP_OK) return st;
  return enqueue_sort(d_in, d_out, n, P, d_splitters, ws, L, s);
}

ap_status ap_sort_u32_ws(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_splitters,
                         void* d_ws, size_t ws_bytes, void* stream) {
  ApRange range("ap_sort_u32_ws");
  ap_status st = check_sort_args(d_in, d_out, n, P);
  if (st != AP_OK) return st;
  return sort_with_ws(d_in, d_out, n, P, d_splitters, d_ws, ws_bytes, static_cast<hipStream_t>(stream));
}

size_t ap_sort_pairs_workspace_bytes(size_t n) {
  if (n >= AP_MAX_KEYS) return 0;
  return layout_for(n, true).total;
}

ap_status ap_sort_pairs_u32(const uint32_t* d_keys_in, const uint32_t* d_vals_in, uint32_t* d_keys_out,
                            uint32_t* d_vals_out, size_t n, int P, uint32_t* d_splitters, void* stream) {
  ApRange range("ap_sort_pairs_u32");
  ap_status st = check_pairs_args(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, P);
  if (st != AP_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) return pairs_with_ws(nullptr, nullptr, nullptr, nullptr, 0, P, d_splitters, nullptr, 0, s);
  const Layout L = layout_for(n, true);
  void* ws = nullptr;
  st = cached_workspace(L.total, s, &ws);
  if (st != AP_OK) return st;
  return enqueue_sort(d_keys_in, d_keys_out, n, P, d_splitters, ws, L, s, d_vals_in, d_vals_out);
}

ap_status ap_sort_pairs_u32_ws(const uint32_t* d_keys_in, const uint32_t* d_vals_in, uint32_t* d_keys_out,
                               uint32_t* d_vals_out, size_t n, int P, uint32_t* d_splitters, void* d_ws,
                               size_t ws_bytes, void* stream) {
  ApRange range("ap_sort_pairs_u32_ws");
  ap_status st = check_pairs_args(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, P);
  if (st != AP_OK) return st;
  return pairs_with_ws(d_keys_in, d_vals_in, d_keys_out, d_vals_out, n, P, d_splitters, d_ws, ws_bytes,
                       static_cast<hipStream_t>(stream));
}

ap_status ap_digit_plan_u32(const uint32_t* d_in, size_t n, int digit_bits, uint32_t* d_hist, uint32_t* d_plan,
                            void* stream) {
  ApRange range("ap_digit_plan_u32");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (digit_bits < 4 || digit_bits > 11) return fail(AP_ERR_INVALID, "digit_bits must be in [4, 11]");
  if (n >= AP_MAX_KEYS) return fail(AP_ERR_INVALID, "n must be < 2^30");
  if (!d_hist) return fail(AP_ERR_INVALID, "d_hist is NULL");
  if (n && (!d_in || ((uintptr_t)d_in & 3u))) return fail(AP_ERR_INVALID, "bad key pointer");
  return enqueue_digit_plan(d_in, n, digit_bits, d_hist, d_plan, s);
}

ap_status ap_release_cache(void) { return release_cache(); }

int ap_rank_check_state(void) { return lane_order_state(); }

ap_status ap_set_rank_mode(int mode) {
  if (mode != 0 && mode != 1) return fail(AP_ERR_INVALID, "rank mode must be 0 (auto) or 1 (match)");
  set_rank_mode(mode);
  return AP_OK;
}

ap_status ap_debug_pass(int mode, uint64_t seed, unsigned long long* d_trace, size_t trace_records) {
  if (mode < PASS_DBG_NONE || mode > PASS_DBG_TRACE) return fail(AP_ERR_INVALID, "debug mode must be 0, 1 or 2");
  if (mode == PASS_DBG_TRACE && (!d_trace || trace_records == 0))
    return fail(AP_ERR_INVALID, "the trace mode needs a trace buffer");
  if (((uintptr_t)d_trace) & 7u) return fail(AP_ERR_INVALID, "trace buffer must be 8-byte aligned");
  std::lock_guard<std::mutex> lk(g_dbg_mu);
  g_dbg = PassDebugState{mode, seed, mode == PASS_DBG_TRACE ? d_trace : nullptr,
                         mode == PASS_DBG_TRACE ? (uint64_t)trace_records : 0u};
  return AP_OK;
}

ap_status ap_set_pass_shape(int shape) {
  if (shape < -1 || shape > 3) return fail(AP_ERR_INVALID, "shape must be -1 (by size) or 0..3");
  g_shape_override.store(shape);
  return AP_OK;
}

}  // extern "C"
