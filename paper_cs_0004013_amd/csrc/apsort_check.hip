// ap_check_u32 / ap_check_u32_batch: the result check of a sort, on the device.  The contest
// program of the paper's Sec. 1.1 checked every result it timed; a served sort is checked the same
// way here without moving keys to the host: the output must be in nondecreasing order, and it must
// hold the same multiset of keys as the input, which an order-independent hash of the keys (sum
// and xor of a 64-bit mix of each key) compares.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "apsort.h"
#include "apsort_device.h"
#include "apsort_internal.h"

namespace aps {

// SplitMix64 finaliser (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014): a bijective mix of a 64-bit word.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The workgroups of one grid row sweep k[0..n): a[0] += descents (i with k[i] > k[i+1]),
// a[1] += sum of mix64(k[i]), a[2] ^= xor of mix64(k[i]).
__device__ __forceinline__ void check_range(gptr<const uint32_t> k, size_t n, unsigned long long* a) {
  uint64_t sum = 0, x = 0, bad = 0;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const uint32_t v = k[i];
    const uint64_t h = mix64(v);
    sum += h;
    x ^= h;
    if (i + 1 < n && v > k[i + 1]) ++bad;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off, 64);
    x ^= __shfl_xor(x, off, 64);
    bad += __shfl_xor(bad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (bad) atomicAdd(&a[0], (unsigned long long)bad);
    atomicAdd(&a[1], (unsigned long long)sum);
    atomicXor(&a[2], (unsigned long long)x);
  }
}

__global__ __launch_bounds__(256) void k_check_one(const uint32_t* __restrict__ keys, size_t n,
                                                   unsigned long long* __restrict__ acc) {
  check_range(gmem(keys), n, acc);
}

// Row blockIdx.y checks array keys[y] of counts[y] keys into acc[3y .. 3y+2].
__global__ __launch_bounds__(256) void k_check_batch(const uint32_t* const* __restrict__ keys,
                                                     const uint64_t* __restrict__ counts,
                                                     unsigned long long* __restrict__ acc) {
  // the array pointer is read from memory: global view, so that the loads are not flat
  check_range(gmem(keys[blockIdx.y]), counts[blockIdx.y], acc + 3 * (size_t)blockIdx.y);
}

static unsigned check_blocks(size_t n) {
  const size_t b = (n + 256 * 16 - 1) / (256 * 16);
  return (unsigned)std::max<size_t>(1, std::min<size_t>(b, (size_t)4 * device_cus()));
}

}  // namespace aps

using namespace aps;

extern "C" {

ap_status ap_check_u32(const uint32_t* d_keys, size_t n, uint64_t* d_acc, void* stream) {
  ApRange range("ap_check_u32");
  if (!d_acc || ((uintptr_t)d_acc & 7u)) return fail(AP_ERR_INVALID, "d_acc must be an 8-byte aligned device pointer");
  if (n && (!d_keys || ((uintptr_t)d_keys & 3u))) return fail(AP_ERR_INVALID, "bad key pointer");
  if (n == 0) return AP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_check_one, dim3(check_blocks(n)), dim3(256), 0, s, d_keys, n,
                     reinterpret_cast<unsigned long long*>(d_acc));
  return check_launch(s, "k_check_one");
}

ap_status ap_check_u32_batch(const uint32_t* const* d_keys, const uint64_t* d_counts, int count, size_t max_n,
                             uint64_t* d_acc, void* stream) {
  ApRange range("ap_check_u32_batch");
  if (count < 0 || count > 65535) return fail(AP_ERR_INVALID, "count must be in [0, 65535]");
  if (count == 0) return AP_OK;
  if (!d_keys || !d_counts || !d_acc || (((uintptr_t)d_keys | (uintptr_t)d_counts | (uintptr_t)d_acc) & 7u))
    return fail(AP_ERR_INVALID, "d_keys, d_counts and d_acc must be 8-byte aligned device pointers");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_check_batch, dim3(check_blocks(max_n), (unsigned)count), dim3(256), 0, s, d_keys, d_counts,
                     reinterpret_cast<unsigned long long*>(d_acc));
  return check_launch(s, "k_check_batch");
}

}  // extern "C"
