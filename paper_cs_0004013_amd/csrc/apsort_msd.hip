// ap_sort_u32_msd: the sort organised as the paper's phases instead of a least-significant-digit
// sort over every digit: the keys are first bucketed on their high-order bits (Sec. 3.2: buckets
// are the values of the top bits, 4096 and later 8192 of them, Sec. 4.7), and every bucket is then
// sorted on its own by a local radix sort (Sec. 3.3, 3.3.1).  On one GPU:
//   1. bucketing: the two high-order 8-bit digits (bits 16..31) through the device-wide stable
//      digit passes of the single-array sort, so the output holds the keys ordered by their top
//      16 bits, buckets of equal top bits contiguous and in bucket order (2^16 buckets);
//   2. the bucket boundaries by binary search in that output;
//   3. the local sorts: the batched segmented sort of the buckets in place (digits 2 and 3 are
//      constant inside a bucket and skipped; short buckets are sorted by one workgroup in LDS,
//      buckets of 2^20 keys or more by device-wide passes);
//   4. the P-1 splitters of the sorted output.
// The bucketing is two passes and not one scatter on 12-13 bits: a digit pass keeps per-wave
// counters of every bucket and a tile of keys in LDS, which leaves room for 2^8 buckets, and one
// scatter into 2^12-2^13 buckets would write runs of one to eight keys per tile.
#include <hip/hip_runtime.h>

#include "apsort.h"
#include "apsort_device.h"
#include "apsort_internal.h"

namespace aps {

constexpr uint32_t kMsdBuckets = 1u << 16;  // values of the top 16 bits

// offsets[u] = number of keys whose top 16 bits are below u (u = 0..2^16; offsets[2^16] = n), by
// binary search in keys ordered by their top 16 bits.  Thread 0 also marks the plan's sorted keys
// as being in the output with nothing to copy, for the splitters that follow the local sorts.
__global__ __launch_bounds__(256) void k_msd_bounds(const uint32_t* __restrict__ keys, uint32_t n,
                                                   uint32_t* __restrict__ offsets, uint32_t* __restrict__ plan) {
  const uint32_t u = blockIdx.x * 256 + threadIdx.x;
  if (u > kMsdBuckets) return;
  uint32_t lo = 0, hi = n;
  if (u < kMsdBuckets) {
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo) / 2;
      if ((keys[mid] >> 16) < u) lo = mid + 1;
      else hi = mid;
    }
  } else {
    lo = n;
  }
  offsets[u] = lo;
  if (u == 0) {
    plan[PL_FINAL] = SEL_OUT;
    plan[PL_COPY] = 0u;
  }
}

static size_t up256m(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace aps

using namespace aps;

extern "C" {

ap_status ap_sort_u32_msd(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_splitters,
                          void* stream) {
  ApRange range("ap_sort_u32_msd");
  ap_status st = check_sort_args(d_in, d_out, n, P);
  if (st != AP_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) return (P > 1 && d_splitters) ? fill_u32(d_splitters, 0xFFFFFFFFu, (size_t)P - 1, s) : AP_OK;
  const Layout L = layout_for(n);
  void* ws = nullptr;
  st = cached_workspace(L.total + up256m(sizeof(uint32_t) * (kMsdBuckets + 1)), s, &ws);
  if (st != AP_OK) return st;
  char* w = static_cast<char*>(ws);
  uint32_t* plan = reinterpret_cast<uint32_t*>(w + L.plan);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(w + L.tmp);
  uint32_t* offsets = reinterpret_cast<uint32_t*>(w + L.total);
  // 1. bucketing on the top two digits; the keys end in d_out ordered by their top 16 bits
  st = enqueue_sort(d_in, d_out, n, 1, nullptr, ws, L, s, nullptr, nullptr, 2);
  if (st != AP_OK) return st;
  // 2. bucket boundaries
  hipLaunchKernelGGL(k_msd_bounds, dim3((kMsdBuckets + 1 + 255) / 256), dim3(256), 0, s, d_out, (uint32_t)n, offsets,
                     plan);
  st = check_launch(s, "k_msd_bounds");
  if (st != AP_OK) return st;
  // 3. local sort of every bucket, in place
  st = ap_sort_u32_segmented(d_out, n, offsets, (int)kMsdBuckets, nullptr, stream);
  if (st != AP_OK) return st;
  // 4. splitters of the sorted keys
  if (P > 1 && d_splitters) {
    st = enqueue_finalize(d_in, d_out, tmp, n, plan, P, d_splitters, s);
  }
  return st;
}

}  // extern "C"
