// Internal declarations shared by the host translation units of libapsort.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "apsort.h"

namespace aps {

// Byte offsets of the single-array sort workspace (see layout_for).
struct Layout {
  size_t hist, base, plan, done, tctr, status, tmp, total;
  size_t zero_bytes;  // bytes from tctr that k_hist_plan clears on every call
  size_t init_bytes;  // bytes from 0 that must be zero before the first call
  uint32_t ntiles;
  int tile_keys;
};

Layout layout_for(size_t n);

ap_status fail(ap_status st, const char* fmt, ...);
ap_status hip_fail(hipError_t e, const char* what);
ap_status check_launch(hipStream_t s, const char* what);
int device_cus();
bool lane_order_ok();
ap_status check_lane_order(hipStream_t s);
ap_status fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s);
// Kernel timing: prof_begin/prof_end bracket one launch when profiling is on for this thread.
void prof_begin(int kind, hipStream_t s);
void prof_end(hipStream_t s);

ap_status enqueue_digit_plan(const uint32_t* d_in, size_t n, int bits, uint32_t* d_hist, uint32_t* d_plan,
                             hipStream_t s);

}  // namespace aps
