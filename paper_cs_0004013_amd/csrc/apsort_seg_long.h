// Device-wide passes over the long segments of a batched sort.
//
// A segment too long for one workgroup is sorted the way the single array is: bucket counts of all
// digits (Sec. 3.2), cumulative totals, then one device-wide pass per non-constant digit, low digit
// first (Sec. 3.3.1), each pass ranking, scanning with decoupled look-back and scattering tile by
// tile (pass_tile).  All long segments of a batch share one flat tile space: segment s owns flat
// tiles [first_tile, first_tile + ntiles), the look-back of a tile stops at its segment's first
// tile, and the workgroups of a pass take flat tiles in increasing order from one counter per
// pass, so tiles of all long segments are in flight together.  Keys are sorted in place through
// the segment's scratch; an odd number of passes ends with a copy back.
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

// Bucket counts of every 8-bit digit of every long segment, and zeroed look-back words for every
// flat tile.  Workgroup w takes a contiguous range of flat tiles (tiles of one segment are mostly
// counted by few workgroups), counts into wave-private LDS counters and adds them to the segment's
// global counts whenever its range leaves a segment.
template <int TILE>
__global__ __launch_bounds__(1024) void k_seg_long_hist(const SegCtl* __restrict__ ctl,
                                                       const LongSeg* __restrict__ longs,
                                                       uint32_t* __restrict__ hist, uint32_t* __restrict__ status,
                                                       size_t status_pass_words) {
  constexpr int HW = 4 * 256;
  __shared__ uint32_t h[16 * HW];  // one copy per wave
  const unsigned long long cur = ld_agent_u64(&ctl->long_cursor);
  const uint32_t nlong = (uint32_t)(cur >> 32), ntiles = (uint32_t)cur;
  if (ntiles == 0u) return;
  const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const uint32_t f0 = blockIdx.x * per;
  const uint32_t f1 = min(f0 + per, ntiles);
  if (f0 >= f1) return;
  const int tid = threadIdx.x, wid = tid >> 6;
  for (int i = tid; i < 16 * HW; i += 1024) h[i] = 0u;
  // look-back words of this range's tiles, all four passes
  for (int d = 0; d < 4; ++d) {
    uint4* z = reinterpret_cast<uint4*>(status + (size_t)d * status_pass_words + (size_t)f0 * 256);
    for (uint32_t i = tid; i < (f1 - f0) * 64u; i += 1024) z[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  __syncthreads();
  uint32_t* hw = h + wid * HW;
  uint32_t slot = long_slot(longs, nlong, f0);
  uint32_t f = f0;
  while (f < f1) {
    const LongSeg ls = longs[slot];
    const uint32_t last = min(f1, ls.first_tile + ls.ntiles);
    const uint32_t k0 = (f - ls.first_tile) * (uint32_t)TILE;
    const uint32_t k1 = min(ls.n, (last - ls.first_tile) * (uint32_t)TILE);
    for (uint32_t i = k0 + tid; i < k1; i += 1024) {
      const uint32_t key = ls.keys[i];
#pragma unroll
      for (int d = 0; d < 4; ++d) atomicAdd(&hw[d * 256 + ((key >> (8 * d)) & 255u)], 1u);
    }
    __syncthreads();
    uint32_t* g = hist + (size_t)slot * HW;
    for (int j = tid; j < HW; j += 1024) {
      uint32_t c = 0u;
#pragma unroll
      for (int w = 0; w < 16; ++w) {
        c += h[w * HW + j];
        h[w * HW + j] = 0u;
      }
      if (c) add_agent(&g[j], c);
    }
    __syncthreads();
    f = last;
    ++slot;
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

// One digit pass over the flat tiles of all long segments: workgroup b (b < number of flat
// tiles; the others exit at once) takes the next flat tile from the pass's counter, so tiles start
// in increasing order and a look-back only waits on tiles already running.  A tile of a segment
// whose digit is constant is skipped (the whole segment skips the pass, so no tile of it is
// looked back at).
template <int WAVES, int IPT, int RANK>
__global__ __launch_bounds__(WAVES * 64) void k_seg_long_pass(SegCtl* __restrict__ ctl, const LongSeg* __restrict__ longs,
                                                             const uint32_t* __restrict__ base,
                                                             uint32_t* __restrict__ status, int d) {
  __shared__ PassSmem<8, WAVES, IPT, RANK, false> sm;
  const unsigned long long cur = ld_agent_u64(&ctl->long_cursor);
  const uint32_t nlong = (uint32_t)(cur >> 32), ntiles = (uint32_t)cur;
  if (blockIdx.x >= ntiles) return;
  if (threadIdx.x == 0) {
    const uint32_t f = add_agent(&ctl->long_ctr[d], 1u);
    sm.tile = f;
    sm.aux[0] = long_slot(longs, nlong, f);
  }
  pass_clear(sm);
  __syncthreads();
  const uint32_t f = sm.tile, slot = sm.aux[0];
  const LongSeg& ls = longs[slot];
  if (!ls.run[d]) return;
  const uint32_t* src = ls.rd_tmp[d] ? ls.tmp : ls.keys;
  uint32_t* dst = ls.rd_tmp[d] ? ls.keys : ls.tmp;
  pass_tile<8, WAVES, IPT, RANK, 4, false>(sm, src, dst, nullptr, nullptr, ls.n, f - ls.first_tile, 8 * d,
                                           base + (size_t)slot * 1024 + d * 256, status + (size_t)ls.first_tile * 256);
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
    for (uint32_t i = k0 + threadIdx.x; i < k1; i += 256) ls.keys[i] = ls.tmp[i];
  }
}

}  // namespace aps
