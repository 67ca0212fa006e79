// ap_sort_u32_noalloc: the single-array sort with its scratch in a fixed device array of this
// library instead of allocated memory, for callers that cannot allocate (code under graph
// capture, serving loops, harnesses that forbid allocation).
//
// The array lives in device memory of every GPU the library runs on until the process ends.  In
// host code its name is only a host-side handle, so the device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and that address, never the name, is
// what the launches get.  Every call on one device shares the array: calls that overlap in time on
// one device race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "apsort.h"
#include "apsort_internal.h"

namespace aps {

// Workspace of the largest accepted sort (AP_NOALLOC_MAX_KEYS keys): control block 133 KiB,
// look-back status <= 4 MiB (4 passes x 1024 tiles of the smallest 4K-key shape x 256 buckets),
// ping-pong buffer 16 MiB.  layout_for() is checked against this size on every call.
constexpr size_t kNoAllocScratchBytes = (size_t)26 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_na_mu;
static std::vector<void*> g_na_ptr;  // per device: device address of `scratch`, null until looked up

static ap_status noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_na_mu);
  if ((int)g_na_ptr.size() <= dev) g_na_ptr.resize(dev + 1, nullptr);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255u)) return fail(AP_ERR_HIP, "scratch array has no usable device address");
    g_na_ptr[dev] = p;
  }
  *out = g_na_ptr[dev];
  return AP_OK;
}

}  // namespace aps

using namespace aps;

extern "C" {

ap_status ap_sort_u32_noalloc(const uint32_t* d_in, uint32_t* d_out, size_t n, int P, uint32_t* d_splitters,
                              void* stream) {
  ApRange range("ap_sort_u32_noalloc");
  ap_status st = check_sort_args(d_in, d_out, n, P);
  if (st != AP_OK) return st;
  if (n > AP_NOALLOC_MAX_KEYS)
    return fail(AP_ERR_INVALID, "n = %zu exceeds the no-allocation maximum of %zu keys", n,
                (size_t)AP_NOALLOC_MAX_KEYS);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n == 0) return (P > 1 && d_splitters) ? fill_u32(d_splitters, 0xFFFFFFFFu, (size_t)P - 1, s) : AP_OK;
  const Layout L = layout_for(n);
  if (L.total > kNoAllocScratchBytes)
    return fail(AP_ERR_INVALID, "sort of %zu keys needs %zu scratch bytes, the fixed array holds %zu", n, L.total,
                kNoAllocScratchBytes);
  void* ws = nullptr;
  st = noalloc_scratch(&ws);
  if (st != AP_OK) return st;
  // The array keeps whatever the previous call left: zero the control words that must start at
  // zero (bucket-count copies, totals, plan, completion counter) with a kernel, not a memset, so
  // that the call can be captured into a graph.
  st = fill_u32(static_cast<uint32_t*>(ws), 0u, L.init_bytes / 4, s);
  if (st != AP_OK) return st;
  return enqueue_sort(d_in, d_out, n, P, d_splitters, ws, L, s);
}

}  // extern "C"
