// Device-wide passes over the long segments of a batched sort.
//
// A segment too long for one workgroup is sorted the way the single array is: bucket counts of all
// digits (Sec. 3.2), cumulative totals, then one device-wide pass per non-constant digit, low digit
// first (Sec. 3.3.1), each pass ranking, scanning with decoupled look-back and scattering tile by
// tile (pass_tile).  All long segments of a batch share one flat tile space: segment s owns flat
// tiles [first_tile, first_tile + ntiles), the look-back of a tile stops at its segment's first
// tile, and the persistent workgroups of a pass take flat tiles in increasing order from one
// counter per pass, so tiles of all long segments are in flight together.  Keys are sorted in
// place through the segment's scratch; an odd number of passes ends with a copy back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apsort_device.h"
#include "apsort_pass_core.h"
#include "apsort_seg_types.h"

namespace aps {

// Slot of the long segment owning flat tile f: the last slot whose first tile is <= f.
__device__ __forceinline__ uint32_t long_slot(const LongSeg* __restrict__ longs, uint32_t nlong, uint32_t f) {
  uint32_t lo = 0, hi = nlong;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (longs[mid].first_tile <= f) lo = mid;
    else hi = mid;
  }
  return lo;
}
// The same search over the first tiles cached in LDS.
__device__ __forceinline__ uint32_t long_slot_lds(const uint32_t* first, uint32_t nlong, uint32_t f) {
  uint32_t lo = 0, hi = nlong;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (first[mid] <= f) lo = mid;
    else hi = mid;
  }
  return lo;
}
constexpr uint32_t kLongSlotCache = 512;  // first tiles of up to this many long segments kept in LDS

// Bucket counts of every 8-bit digit of every long segment, and zeroed look-back words for every
// flat tile.  Workgroup w takes a contiguous range of flat tiles (tiles of one segment are mostly
// counted by few workgroups).  As in k_hist_plan, every lane position l of the wave owns a private
// copy of the 1024 counters (4 digits x 256) as 16-bit halves: bucket B is half B & 1 of LDS word
// (B / 2) * 64 + l, so the 64 lanes of one atomic add hit 64 different banks whatever the keys.  A
// copy counts the keys of 16 threads; the copies are summed into the segment's global counts when
// the range leaves a segment and after every kLongHistFlush tiles, so that a copy counts at most
// 16 * kLongHistFlush * TILE / 1024 < 2^16 keys.
constexpr uint32_t kLongHistFlush = 32;
template <int TILE>
__global__ __launch_bounds__(1024) void k_seg_long_hist(const SegCtl* __restrict__ ctl,
                                                       const LongSeg* __restrict__ longs,
                                                       uint32_t* __restrict__ hist, uint32_t* __restrict__ status,
                                                       size_t status_pass_words) {
  static_assert(16u * kLongHistFlush * (TILE / 1024) < 65536u, "16-bit lane counters would overflow");
  __shared__ uint32_t h[512 * 64];  // 1024 16-bit counters per lane position
  const unsigned long long cur = ld_agent_u64(&ctl->long_cursor);
  const uint32_t nlong = (uint32_t)(cur >> 32), ntiles = (uint32_t)cur;
  if (ntiles == 0u) return;
  const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const uint32_t f0 = blockIdx.x * per;
  const uint32_t f1 = min(f0 + per, ntiles);
  if (f0 >= f1) return;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  for (uint32_t i = tid; i < 512u * 64u; i += 1024u) h[i] = 0u;
  // look-back words of this range's tiles, all four passes
  for (int d = 0; d < 4; ++d) {
    uint4* z = reinterpret_cast<uint4*>(status + (size_t)d * status_pass_words + (size_t)f0 * 256);
    for (uint32_t i = tid; i < (f1 - f0) * 64u; i += 1024u) z[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  __syncthreads();
  uint32_t* hc = h + lane;
  auto count = [&](uint32_t key) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const uint32_t b = (uint32_t)(d * 256) + ((key >> (8 * d)) & 255u);
      atomicAdd(&hc[(b >> 1) * 64u], 1u << ((b & 1u) * 16u));
    }
  };
  uint32_t slot = long_slot(longs, nlong, f0);
  uint32_t f = f0;
  while (f < f1) {
    const LongSeg ls = longs[slot];
    const uint32_t seg_end = ls.first_tile + ls.ntiles;
    const uint32_t last = min(min(f1, seg_end), f + kLongHistFlush);
    const uint32_t k0 = (f - ls.first_tile) * (uint32_t)TILE;
    const uint32_t k1 = min(ls.n, (last - ls.first_tile) * (uint32_t)TILE);
    const gptr<const uint32_t> keys = gmem(ls.keys);
    uint32_t i = k0 + tid;
    for (; i + 3u * 1024u < k1; i += 4u * 1024u) {
      const uint32_t a0 = keys[i], a1 = keys[i + 1024u], a2 = keys[i + 2048u], a3 = keys[i + 3072u];
      count(a0); count(a1); count(a2); count(a3);
    }
    for (; i < k1; i += 1024u) count(keys[i]);
    __syncthreads();
    uint32_t* g = hist + (size_t)slot * 1024;
    for (uint32_t j = tid; j < 1024u; j += 1024u) {
      // lane copies read in a rotated order: the 64 lanes of a read hit 64 different banks
      const uint32_t row = (j >> 1) * 64u, sh = (j & 1u) * 16u;
      uint32_t c = 0u;
#pragma unroll 16
      for (uint32_t q = 0; q < 64u; ++q) c += (h[row + ((q + j) & 63u)] >> sh) & 0xFFFFu;
      if (c) add_agent(&g[j], c);
    }
    __syncthreads();
    for (uint32_t x = tid; x < 512u * 64u; x += 1024u) h[x] = 0u;
    __syncthreads();
    f = last;
    if (f == seg_end) ++slot;
  }
}

// Plan of each long segment from its bucket counts: which digit passes run, their buffers, and the
// cumulative totals per digit.
__global__ __launch_bounds__(256) void k_seg_long_plan(const SegCtl* __restrict__ ctl, LongSeg* __restrict__ longs,
                                                      const uint32_t* __restrict__ hist, uint32_t* __restrict__ base) {
  __shared__ uint32_t s_h[4 * 256];
  __shared__ uint32_t s_const[4];
  __shared__ uint32_t s_scan[4];
  const uint32_t nlong = (uint32_t)(ld_agent_u64(&ctl->long_cursor) >> 32);
  const int tid = threadIdx.x;
  for (uint32_t s = blockIdx.x; s < nlong; s += gridDim.x) {
    const uint32_t* g = hist + (size_t)s * 1024;
    const uint32_t n = longs[s].n;
    if (tid < 4) s_const[tid] = 0u;
    __syncthreads();
    for (int j = tid; j < 1024; j += 256) {
      const uint32_t c = g[j];
      s_h[j] = c;
      if (c == n) s_const[j >> 8] = 1u;  // one bucket holds every key: the digit is constant
    }
    for (int d = 0; d < 4; ++d) lds_exclusive_scan<256, 256>(s_h + d * 256, s_scan);
    for (int j = tid; j < 1024; j += 256) base[(size_t)s * 1024 + j] = s_h[j];
    if (tid == 0) {
      // in place: the first pass that runs reads the keys and writes the scratch, then they alternate
      uint32_t npass = 0, in_tmp = 0;
      for (int d = 0; d < 4; ++d) {
        const uint32_t run = s_const[d] ? 0u : 1u;
        longs[s].run[d] = run;
        longs[s].rd_tmp[d] = in_tmp;
        if (run) {
          in_tmp ^= 1u;
          ++npass;
        }
      }
      longs[s].npass = npass;
      longs[s].final_tmp = in_tmp;
    }
    __syncthreads();
  }
}

// One digit pass over the flat tiles of all long segments.  Persistent (one workgroup per CU, so
// that an empty pass costs a few hundred workgroups, not one per possible tile): every workgroup
// takes the next flat tile from the pass's counter until none is left, so tiles start in
// increasing order and a look-back only waits on tiles already taken by running workgroups, which
// each process one tile at a time.  A tile of a segment whose digit is constant is skipped (the
// whole segment skips the pass, so no tile of it is looked back at).  NT_STORE: the scatter's
// store hint (plain for the passes before the last, as in the single-array sort of large arrays).
template <int WAVES, int IPT, int RANK, bool NT_STORE>
__global__ __launch_bounds__(WAVES * 64) void k_seg_long_pass(SegCtl* __restrict__ ctl, const LongSeg* __restrict__ longs,
                                                             const uint32_t* __restrict__ base,
                                                             uint32_t* __restrict__ status, int d) {
  AP_PASS_SMEM(sm, 8, WAVES, IPT, RANK, false);
  __shared__ uint32_t s_tile, s_slot;
  __shared__ uint32_t s_first[kLongSlotCache];
  const unsigned long long cur = ld_agent_u64(&ctl->long_cursor);
  const uint32_t nlong = (uint32_t)(cur >> 32), ntiles = (uint32_t)cur;
  if (ntiles == 0u) return;
  // the segments' first tiles in LDS: a tile's segment is then found without global round trips
  // (the first barrier of the loop orders these writes before any search)
  const bool cached = nlong <= kLongSlotCache;
  if (cached)
    for (uint32_t s = threadIdx.x; s < nlong; s += WAVES * 64) s_first[s] = longs[s].first_tile;
#pragma unroll 1
  while (true) {
    if (threadIdx.x == 0) {
      const uint32_t f = add_agent(&ctl->long_ctr[d], 1u);
      s_tile = f;
      s_slot = f >= ntiles ? 0u : cached ? long_slot_lds(s_first, nlong, f) : long_slot(longs, nlong, f);
    }
    pass_clear(sm);
    __syncthreads();
    const uint32_t f = s_tile, slot = s_slot;
    if (f >= ntiles) break;
    const LongSeg& ls = longs[slot];
    if (ls.run[d]) {
      const uint32_t rd = ls.rd_tmp[d];
      // an opaque copy of the thread index: see pass_tile
      int tid = (int)threadIdx.x;
      asm volatile("" : "+v"(tid));
      pass_tile<8, WAVES, IPT, RANK, 4, false, PASS_DBG_NONE, NT_STORE>(
          sm, rd ? ls.tmp : ls.keys, rd ? ls.keys : ls.tmp, nullptr, nullptr, ls.n, f - ls.first_tile, 8 * d,
          base + (size_t)slot * 1024 + d * 256, status + (size_t)ls.first_tile * 256, tid);
    }
    __syncthreads();  // every thread is done with this tile's LDS before the next claim
  }
}

// Copy back: the segments whose sorted keys ended in their scratch (an odd number of passes).
template <int TILE>
__global__ __launch_bounds__(256) void k_seg_long_copy(const SegCtl* __restrict__ ctl,
                                                      const LongSeg* __restrict__ longs) {
  const unsigned long long cur = ld_agent_u64(&ctl->long_cursor);
  const uint32_t nlong = (uint32_t)(cur >> 32), ntiles = (uint32_t)cur;
  for (uint32_t f = blockIdx.x; f < ntiles; f += gridDim.x) {
    const uint32_t slot = long_slot(longs, nlong, f);
    const LongSeg& ls = longs[slot];
    if (!ls.final_tmp) continue;
    const uint32_t k0 = (f - ls.first_tile) * (uint32_t)TILE;
    const uint32_t k1 = min(ls.n, k0 + (uint32_t)TILE);
    const gptr<uint32_t> keys = gmem(ls.keys), tmp = gmem(ls.tmp);
    for (uint32_t i = k0 + threadIdx.x; i < k1; i += 256) keys[i] = tmp[i];
  }
}

}  // namespace aps
