// Merge of two sorted runs: the merge step of the merge-exchange (Weaver & Lynes, Sec. 3.4: two
// sorted lists merged in the classic manner, the lower cell keeping the lower values; Sec. 4.6:
// two sorted runs of one array merged in blocks).  On one GPU the merged list is written once and
// the cells' halves are positional slices of it.
//
// Merge path: output position d of the merge of a (na keys) and b (nb keys), ties taking a first,
// is preceded by exactly split(d) keys of a, the smallest i in [max(0, d - nb), min(d, na)] with
// NOT (a[i] <= b[d - 1 - i]).  k_merge_partition finds split() at every 64th tile boundary, then
// at every tile boundary inside those windows (a group of 64, then of 8, lanes per boundary,
// one candidate per lane and round trip; split() is monotone in d); k_merge_tile then merges one tile of T outputs from the
// two sub-runs it owns, staged in LDS, each thread merging IPT consecutive outputs after its own
// search, and writes the tile out coalesced.  Algorithmic bytes: 8 per output key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <vector>

#include "apsort.h"
#include "apsort_internal.h"

namespace aps {

constexpr int kMergeThreads = 512;
constexpr int kMergeIpt = 16;
constexpr uint32_t kMergeTile = kMergeThreads * kMergeIpt;  // 8192 outputs per workgroup

// Number of keys of a among the first d outputs (ties: a first), known to lie in [lo, hi].
// Evaluated by a group of G lanes of one wave (each group its own diagonal d): each round trip
// tests G evenly spaced candidates; the predicate a[i] <= b[d-1-i] is true for a prefix of the
// candidates, so the population count of the group's ballot bits narrows the range G-fold.  A
// wider group needs fewer dependent round trips but gathers more cache lines per search.
// `active` is uniform within a group; the loop runs until every group of the wave is done.
template <int G>
__device__ uint32_t merge_split_group(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, uint32_t d,
                                      uint32_t lo, uint32_t hi, bool active) {
  static_assert(G >= 2 && G <= 64 && (G & (G - 1)) == 0, "group of 2..64 lanes");
  const uint32_t lane = threadIdx.x & 63u, sub = lane & (uint32_t)(G - 1);
  const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << (lane & ~(uint32_t)(G - 1));
  for (;;) {
    const bool more = active && hi - lo > (uint32_t)G;
    if (__ballot(more) == 0ull) break;
    const uint32_t span = hi - lo;
    const uint32_t m = lo + (uint32_t)(((uint64_t)span * sub) / (uint32_t)G);  // m < hi
    const bool p = more && a[m] <= b[d - 1u - m];
    const uint32_t c = (uint32_t)__popcll(__ballot(p) & gmask);
    if (more) {
      const uint32_t m_last_true = lo + (uint32_t)(((uint64_t)span * (c - 1u)) / (uint32_t)G);
      const uint32_t m_first_false = lo + (uint32_t)(((uint64_t)span * c) / (uint32_t)G);
      if (c > 0u) lo = m_last_true + 1u;
      if (c < (uint32_t)G) hi = m_first_false;
    }
  }
  // at most G candidates left: lane `sub` of the group tests lo + sub
  const uint32_t m = lo + sub;
  const bool p = active && m < hi && a[m] <= b[d - 1u - m];
  return lo + (uint32_t)__popcll(__ballot(p) & gmask);
}

// splits[t] = split(min(t * step, n)) for t < nsplits, one group of G lanes per entry.  With
// `coarse` (splits of every ratio-th entry's diagonal, ncoarse of them) each search starts inside
// its coarse window: the split is monotone in the diagonal.
template <int G>
__global__ __launch_bounds__(256) void k_merge_partition(const uint32_t* __restrict__ a, uint32_t na,
                                                         const uint32_t* __restrict__ b, uint32_t nb,
                                                         uint32_t* __restrict__ splits, uint32_t nsplits,
                                                         uint32_t step, const uint32_t* __restrict__ coarse,
                                                         uint32_t ratio, uint32_t ncoarse) {
  const uint32_t t = (blockIdx.x * 256u + threadIdx.x) / (uint32_t)G;
  if (blockIdx.x * 256u + (threadIdx.x & ~63u) >= nsplits * (uint32_t)G) return;  // whole wave past the end
  const bool active = t < nsplits;
  const uint64_t n = (uint64_t)na + nb;
  const uint32_t d = active ? (uint32_t)std::min<uint64_t>((uint64_t)t * step, n) : 0u;
  uint32_t lo = d > nb ? d - nb : 0u;
  uint32_t hi = d < na ? d : na;
  if (coarse && active) {
    const uint32_t c = t / ratio;
    lo = std::max(lo, coarse[c]);
    hi = std::min(hi, coarse[std::min(c + 1u, ncoarse - 1u)]);
  }
  const uint32_t s = merge_split_group<G>(a, b, d, lo, hi, active);
  if (active && (threadIdx.x & (uint32_t)(G - 1)) == 0u) splits[t] = s;
}

// Same search on LDS runs, by one thread (ties: a first).
__device__ __forceinline__ uint32_t merge_split_lds(const uint32_t* sa, uint32_t la, const uint32_t* sb, uint32_t lb,
                                                   uint32_t d) {
  uint32_t lo = d > lb ? d - lb : 0u;
  uint32_t hi = d < la ? d : la;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sa[mid] <= sb[d - 1u - mid]) lo = mid + 1u;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kMergeThreads) void k_merge_tile(const uint32_t* __restrict__ a, uint32_t na,
                                                             const uint32_t* __restrict__ b, uint32_t nb,
                                                             const uint32_t* __restrict__ splits,
                                                             uint32_t* __restrict__ out) {
  constexpr uint32_t T = kMergeTile, PAD = T + T / 32u;
  // the runs, then (after a barrier) the merged tile with one pad word per 32 (fewer bank
  // conflicts); PAD > T, so reading one element past either run stays inside the array
  __shared__ uint32_t s_buf[PAD];
  const uint32_t tid = threadIdx.x, t = blockIdx.x;
  const uint32_t n = na + nb;
  const uint32_t d0 = t * T, d1 = std::min(d0 + T, n);
  const uint32_t i0 = splits[t], i1 = splits[t + 1];
  const uint32_t j0 = d0 - i0, j1 = d1 - i1;
  const uint32_t la = i1 - i0, lb = j1 - j0, len = d1 - d0;
  // fixed trip count, loads first: all of a thread's loads are in flight together.  Runs and
  // output are streamed once, so loads and stores carry the non-temporal hint (~4% faster).
  constexpr int KL = (int)(T / kMergeThreads);
  uint32_t v[KL];
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const uint32_t e = tid + (uint32_t)k * kMergeThreads;
    v[k] = e < la ? __builtin_nontemporal_load(&a[i0 + e])
                  : (e < len ? __builtin_nontemporal_load(&b[j0 + (e - la)]) : 0u);
  }
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const uint32_t e = tid + (uint32_t)k * kMergeThreads;
    if (e < len) s_buf[e] = v[k];
  }
  __syncthreads();
  const uint32_t* sa = s_buf;
  const uint32_t* sb = s_buf + la;
  uint32_t r[kMergeIpt];
  const uint32_t dd = tid * (uint32_t)kMergeIpt;
  if (dd < len) {
    uint32_t i = merge_split_lds(sa, la, sb, lb, dd);
    uint32_t j = dd - i;
    // heads of both runs kept in registers: one LDS read per output
    uint32_t av = sa[i], bv = sb[j];
#pragma unroll
    for (int k = 0; k < kMergeIpt; ++k) {
      // take b only when it is strictly smaller (ties: a first); an exhausted run is never taken
      const bool take_b = j < lb && (i >= la || bv < av);
      r[k] = take_b ? bv : av;
      const uint32_t nv = take_b ? sb[j + 1u] : sa[i + 1u];  // index <= len <= T < PAD
      j += take_b ? 1u : 0u;
      i += take_b ? 0u : 1u;
      bv = take_b ? nv : bv;
      av = take_b ? av : nv;
    }
  }
  __syncthreads();  // every run element has been read
  if (dd < len) {
#pragma unroll
    for (int k = 0; k < kMergeIpt; ++k) {
      const uint32_t e = dd + (uint32_t)k;
      s_buf[e + (e >> 5)] = r[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const uint32_t e = tid + (uint32_t)k * kMergeThreads;
    if (e < len) __builtin_nontemporal_store(s_buf[e + (e >> 5)], &out[d0 + e]);
  }
}

// ------------------------------------------------------------------------- host
struct MergeEntry {
  int dev;
  hipStream_t stream;
  uint32_t* buf;   // partition splits, then (adjacent-run merge) a copy of the runs
  size_t words;
};
static std::mutex g_merge_mu;
static std::vector<MergeEntry> g_merge;

// Scratch of at least `words` u32 for (device, stream); growing synchronises the stream first.
static ap_status merge_scratch(hipStream_t s, size_t words, uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_merge_mu);
  for (auto& c : g_merge) {
    if (c.dev != dev || c.stream != s) continue;
    if (c.words < words) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      (void)hipFree(c.buf);
      c.buf = nullptr;
      c.words = 0;
      e = hipMalloc(&c.buf, words * sizeof(uint32_t));
      if (e != hipSuccess) return hip_fail(e, "hipMalloc(merge scratch)");
      c.words = words;
    }
    *out = c.buf;
    return AP_OK;
  }
  MergeEntry c{dev, s, nullptr, words};
  e = hipMalloc(&c.buf, words * sizeof(uint32_t));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(merge scratch)");
  g_merge.push_back(c);
  *out = c.buf;
  return AP_OK;
}

// Frees the merge scratch of device `dev` (every stream); the caller has synchronised the device.
void release_merge_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_merge_mu);
  std::vector<MergeEntry> keep;
  for (auto& c : g_merge) {
    if (c.dev == dev) (void)hipFree(c.buf);
    else keep.push_back(c);
  }
  g_merge.swap(keep);
}

constexpr uint32_t kMergeRatio = 64;  // tiles per coarse partition window

// scratch words: the tile splits, then the coarse splits
size_t merge_split_words(size_t n) {
  const size_t ntiles = (n + kMergeTile - 1) / kMergeTile;
  return (ntiles + 1) + (ntiles + kMergeRatio - 1) / kMergeRatio + 1;
}

ap_status enqueue_merge(const uint32_t* a, uint32_t na, const uint32_t* b, uint32_t nb, uint32_t* out,
                        uint32_t* splits, hipStream_t s) {
  const uint32_t n = na + nb;
  const uint32_t ntiles = (n + kMergeTile - 1) / kMergeTile;
  const uint32_t ncoarse = (ntiles + kMergeRatio - 1) / kMergeRatio + 1;
  uint32_t* coarse = splits + ntiles + 1;
  prof_begin(AP_KIND_MERGE, s);
  constexpr int kGc = 64, kGf = 8;  // lanes per search: coarse (few, long searches), fine (many, short)
  hipLaunchKernelGGL(k_merge_partition<kGc>, dim3((ncoarse + 256 / kGc - 1) / (256 / kGc)), dim3(256), 0, s, a, na,
                     b, nb, coarse, ncoarse, kMergeTile * kMergeRatio, (const uint32_t*)nullptr, 1u, 0u);
  hipLaunchKernelGGL(k_merge_partition<kGf>, dim3((ntiles + 1 + 256 / kGf - 1) / (256 / kGf)), dim3(256), 0, s, a,
                     na, b, nb, splits, ntiles + 1, kMergeTile, (const uint32_t*)coarse, kMergeRatio, ncoarse);
  hipLaunchKernelGGL(k_merge_tile, dim3(ntiles), dim3(kMergeThreads), 0, s, a, na, b, nb, splits, out);
  prof_end(s);
  return check_launch(s, "k_merge_tile");
}

static bool overlaps(const void* p, size_t np, const void* q, size_t nq) {
  const uintptr_t a0 = (uintptr_t)p, a1 = a0 + np * 4, b0 = (uintptr_t)q, b1 = b0 + nq * 4;
  return np && nq && a0 < b1 && b0 < a1;
}

}  // namespace aps

using namespace aps;

extern "C" {

ap_status ap_merge_u32(const uint32_t* d_a, size_t na, const uint32_t* d_b, size_t nb, uint32_t* d_out,
                       void* stream) {
  ApRange range("ap_merge_u32");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (na >= AP_MAX_KEYS || nb >= AP_MAX_KEYS || na + nb >= AP_MAX_KEYS)
    return fail(AP_ERR_INVALID, "na + nb must be < 2^30");
  if (na + nb == 0) return AP_OK;
  if ((na && !d_a) || (nb && !d_b) || !d_out) return fail(AP_ERR_INVALID, "NULL buffer with a nonzero count");
  if (((uintptr_t)d_a | (uintptr_t)d_b | (uintptr_t)d_out) & 3u)
    return fail(AP_ERR_INVALID, "buffers must be 4-byte aligned");
  if (overlaps(d_out, na + nb, d_a, na) || overlaps(d_out, na + nb, d_b, nb))
    return fail(AP_ERR_INVALID, "the output overlaps an input (use ap_merge_adjacent_u32 for one array)");
  uint32_t* splits = nullptr;
  ap_status st = merge_scratch(s, merge_split_words(na + nb), &splits);
  if (st != AP_OK) return st;
  return enqueue_merge(d_a, (uint32_t)na, d_b, (uint32_t)nb, d_out, splits, s);
}

ap_status ap_merge_adjacent_u32(uint32_t* d_keys, size_t na, size_t nb, void* stream) {
  ApRange range("ap_merge_adjacent_u32");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (na >= AP_MAX_KEYS || nb >= AP_MAX_KEYS || na + nb >= AP_MAX_KEYS)
    return fail(AP_ERR_INVALID, "na + nb must be < 2^30");
  const size_t n = na + nb;
  if (n == 0 || na == 0 || nb == 0) return AP_OK;  // one run: already sorted
  if (!d_keys) return fail(AP_ERR_INVALID, "d_keys is NULL");
  if ((uintptr_t)d_keys & 3u) return fail(AP_ERR_INVALID, "d_keys must be 4-byte aligned");
  const size_t sw = merge_split_words(n);
  uint32_t* scratch = nullptr;
  ap_status st = merge_scratch(s, sw + n + 64, &scratch);
  if (st != AP_OK) return st;
  uint32_t* runs = scratch + (sw + 63) / 64 * 64;  // 256-byte aligned copy of both runs
  hipError_t e = hipMemcpyAsync(runs, d_keys, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(merge runs)");
  return enqueue_merge(runs, (uint32_t)na, runs + na, (uint32_t)nb, d_keys, scratch, s);
}

}  // extern "C"
