// Internal declarations shared by the host translation units of libapsort.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "apsort.h"

namespace aps {

// A roctx range around a library call (named after the entry point), seen by a tracer such as
// rocprofv3 --marker-trace; without a tracer attached the push and pop return at once.
struct ApRange {
  explicit ApRange(const char* name) { roctxRangePushA(name); }
  ~ApRange() { roctxRangePop(); }
  ApRange(const ApRange&) = delete;
  ApRange& operator=(const ApRange&) = delete;
};

// Byte offsets of the single-array sort workspace (see layout_for).
struct Layout {
  size_t hist, base, plan, done, tctr, status, tmp, vtmp, total;
  size_t zero_bytes;  // bytes from tctr that k_hist_plan clears on every call
  size_t init_bytes;  // bytes from 0 that must be zero before the first call
  uint32_t ntiles;
  int tile_keys;
};

Layout layout_for(size_t n, bool pairs = false);

ap_status fail(ap_status st, const char* fmt, ...);
ap_status hip_fail(hipError_t e, const char* what);
ap_status check_launch(hipStream_t s, const char* what);
int device_cus();
bool lane_order_ok();
ap_status check_lane_order(hipStream_t s);
ap_status fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s);
// Frees the merge entry points' cached scratch of device `dev`; the device must be idle.
void release_merge_scratch(int dev);
// Kernel timing: prof_begin/prof_end bracket one launch when profiling is on for this thread.
void prof_begin(int kind, hipStream_t s);
void prof_end(hipStream_t s);
bool prof_active();

// Segmented sort (apsort_seg.hip), shared with the request server.
struct SegDesc;
struct SegCtl;
struct SegGroup {
  int cls_lo, cls_hi, cfg;  // ceil(log2(length)) class range and kernel configuration
};
void launch_seg_group(const SegGroup& g, dim3 grid, hipStream_t s, const SegDesc* order, uint32_t lo, uint32_t hi,
                      int grp, SegCtl* ctl);
int seg_workgroups(const SegGroup& g, uint32_t nwork);
bool seg_group_one_tile(const SegGroup& g);
int seg_tile_keys(int cfg);
void seg_groups(SegGroup* out);  // kSegGroups entries
ap_status seg_groups_check(const SegGroup* grp);  // the used groups partition classes 1..31
void seg_reset(hipStream_t s, SegCtl* ctl);
// d_vout != nullptr: (key, value) pairs, the values read from d_vin and written to d_vout
// (workspace from layout_for(n, true)).
// first_digit > 0: only digits first_digit.. are sorted on (the bucketing variant's high-order
// passes); the output then holds the keys ordered by those digits.
ap_status enqueue_sort(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_spl, void* ws,
                       const Layout& L, hipStream_t s, const uint32_t* d_vin = nullptr, uint32_t* d_vout = nullptr,
                       int first_digit = 0);
// enqueue_sort with the workspace in two pieces: ctl holds the layout's [0, L.init_bytes) (zero
// before the first call and left zero by every call), scratch holds [L.tctr, L.total).
ap_status enqueue_sort_parts(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_spl, void* ctl,
                             void* scratch, const Layout& L, hipStream_t s, const uint32_t* d_vin = nullptr,
                             uint32_t* d_vout = nullptr, int first_digit = 0);
ap_status cached_workspace(size_t need, hipStream_t s, void** out);
// Arrays of at most kSmallSortMax keys: sorted in one launch by one workgroup (apsort_seg.hip).
constexpr uint32_t kSmallSortMax = 16384;
ap_status enqueue_small_sort(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_spl,
                             hipStream_t s);
// k_finalize alone: copy the plan's final buffer into d_out if the plan says so, and the splitters.
ap_status enqueue_finalize(const uint32_t* d_in, uint32_t* d_out, const uint32_t* tmp, size_t n, const uint32_t* plan,
                           int P, uint32_t* d_spl, hipStream_t s);

ap_status check_sort_args(const uint32_t* d_in, const uint32_t* d_out, size_t n, int P);

ap_status enqueue_digit_plan(const uint32_t* d_in, size_t n, int bits, uint32_t* d_hist, uint32_t* d_plan,
                             hipStream_t s);

}  // namespace aps
