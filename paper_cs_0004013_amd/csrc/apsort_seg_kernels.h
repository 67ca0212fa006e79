// Device kernels of the batched segmented sort: many independent key arrays (segments) of one
// buffer, each sorted in place, in one persistent launch.
//
// Each segment is sorted by one workgroup, the way each AP1000 cell runs its own local radix sort
// on the keys it holds (Sec. 3.3 / 3.3.1): a segment that fits in one tile is sorted entirely in
// registers and LDS (read once, written once); a longer one is sorted by the same workgroup with
// one LDS histogram sweep over the segment (Sec. 3.2 bucket counts and cumulative totals for all
// digits) and then, per digit, a sweep over its tiles in order, in which running bucket offsets kept
// in LDS replace any cross-workgroup scan.  Digits constant over a segment are skipped.  Segments
// are taken longest first so the longest ones do not finish last.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apsort.h"
#include "apsort_device.h"
#include "apsort_seg_types.h"

namespace aps {

// Length class ceil(log2(len)) for len >= 2: class c holds lengths in (2^(c-1), 2^c], so a
// configuration whose tile holds 2^c keys sorts every segment of class c in one tile, and
// power-of-two lengths fill their tile exactly.
__device__ __forceinline__ int seg_class(uint32_t len) { return 32 - __clz(len - 1u); }

// Pass 1: validate offsets (off[s] <= off[s+1] <= n_total for every s), count segments per length
// class; the last workgroup turns the counts into a longest-first order of classes, or into an
// empty order when any offset was invalid, and reports the outcome through d_status.  Segments of
// long_min keys or more are not counted: they are sorted by the device-wide passes.
__global__ __launch_bounds__(256) void k_seg_classify(const uint32_t* __restrict__ off, uint32_t nseg,
                                                     uint32_t n_total, uint32_t long_min, SegCtl* __restrict__ ctl,
                                                     uint32_t* __restrict__ d_status) {
  __shared__ uint32_t s_cnt[kSegBuckets];
  __shared__ uint32_t s_bad;
  __shared__ int s_last;
  const uint32_t tid = threadIdx.x;
  if (tid < kSegBuckets) s_cnt[tid] = 0u;
  if (tid == 0) s_bad = 0u;
  __syncthreads();
  for (uint32_t s = blockIdx.x * 256 + tid; s < nseg; s += gridDim.x * 256) {
    const uint32_t a = off[s], b = off[s + 1];
    if (b < a || b > n_total) {
      s_bad = 1u;
      continue;
    }
    const uint32_t len = b - a;
    if (len >= 2 && len < long_min) atomicAdd(&s_cnt[seg_class(len)], 1u);
  }
  __syncthreads();
  if (tid < kSegBuckets && s_cnt[tid]) add_agent(&ctl->count[tid], s_cnt[tid]);
  if (tid == 0 && s_bad) atomicOr(&ctl->bad, 1u);
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    s_last = (add_agent(&ctl->done, 1u) == gridDim.x - 1);
    if (s_last) __threadfence();
  }
  __syncthreads();
  if (!s_last) return;
  if (tid == 0) {
    // Any invalid offset makes segments overlap or leave the buffer: then nothing is sorted.
    const uint32_t bad = ld_agent(&ctl->bad);
    uint32_t run = 0;
    for (int c = kSegBuckets - 1; c >= 0; --c) {  // longest class first
      const uint32_t k = bad ? 0u : ld_agent(&ctl->count[c]);
      ctl->count[c] = k;
      ctl->start[c] = run;
      run += k;
    }
    ctl->nwork = run;
    ctl->done = 0u;
    if (d_status) d_status[0] = bad ? (uint32_t)AP_ERR_INVALID : 0u;
  }
}

// Pass 2: write a descriptor for each valid segment into its class's slots of the work order
// (in place: src == dst == keys + offset, scratch at the same offset of tmp).  A segment of
// long_min keys or more gets a LongSeg slot and a range of flat tiles of long_tile keys instead;
// both come from one 64-bit counter, so flat tile ranges increase with the slot.
// Slots of the work order are claimed once per wave and class: the lanes of a wave whose
// segments share a class take consecutive slots from one atomic add of their count.  (With one
// add per segment, tens of thousands of segments of one class, as the buckets of the bucketing
// sort are, serialize on that class's counter: ~250 us for 32K segments.)
__global__ __launch_bounds__(256) void k_seg_fill(const uint32_t* __restrict__ off, uint32_t nseg, uint32_t n_total,
                                                 uint32_t long_min, uint32_t long_tile, SegCtl* __restrict__ ctl,
                                                 uint32_t* keys, uint32_t* tmp, SegDesc* __restrict__ order,
                                                 LongSeg* __restrict__ longs, uint32_t* __restrict__ long_hist) {
  if (ctl->bad) return;  // invalid offsets: no work
  const int lane = threadIdx.x & 63;
  // the loop bound is uniform over the workgroup, so every lane of a wave takes part in the ballots
  for (uint32_t s0 = blockIdx.x * 256; s0 < nseg; s0 += gridDim.x * 256) {
    const uint32_t s = s0 + threadIdx.x;
    int c = -1;  // class of this lane's short segment, -1 if none
    uint32_t a = 0u, len = 0u;
    if (s < nseg) {
      a = off[s];
      const uint32_t b = off[s + 1];
      if (b >= a && b <= n_total && b - a >= 2u) {
        len = b - a;
        if (len >= long_min) {
          const uint32_t nt = (len + long_tile - 1) / long_tile;
          const unsigned long long got = __hip_atomic_fetch_add(&ctl->long_cursor, (1ull << 32) | nt,
                                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint32_t slot = (uint32_t)(got >> 32);
          LongSeg& ls = longs[slot];
          ls.keys = keys + a;
          ls.tmp = tmp + a;
          ls.n = len;
          ls.first_tile = (uint32_t)got;
          ls.ntiles = nt;
          // The slot's bucket counts start at zero: where they sit in the workspace depends on
          // the call's sizes, so nothing a previous call left there can be trusted.
          uint4* h = reinterpret_cast<uint4*>(long_hist + (size_t)slot * 1024);
          for (int i = 0; i < 256; ++i) h[i] = make_uint4(0u, 0u, 0u, 0u);
        } else {
          c = seg_class(len);
        }
      }
    }
    uint64_t todo = __builtin_amdgcn_ballot_w64(c >= 0);
    while (todo) {
      const int leader = __builtin_ctzll(todo);  // wave-uniform
      const int cl = __builtin_amdgcn_readlane(c, leader);
      const uint64_t same = __builtin_amdgcn_ballot_w64(c == cl);
      uint32_t first = 0u;
      if (lane == leader) first = ctl->start[cl] + add_agent(&ctl->cursor[cl], (uint32_t)__popcll(same));
      first = (uint32_t)__builtin_amdgcn_readlane((int)first, leader);
      if (c == cl) {
        SegDesc dsc;
        dsc.src = keys + a;
        dsc.dst = keys + a;
        dsc.tmp = tmp + a;
        dsc.spl = nullptr;
        dsc.n = len;
        dsc.P = 1u;
        dsc.pad[0] = dsc.pad[1] = 0u;
        order[first + lanes_below(same)] = dsc;
      }
      todo &= ~same;
    }
  }
}

// Shared memory of k_seg_sort.  The histogram copies of the first sweep and the tile buffers of
// the digit sweeps are never live at the same time.
template <int BITS, int WAVES, int IPT, int LCOPIES>
struct SegSmem {
  static constexpr int R = 1 << BITS;
  static constexpr int D = (32 + BITS - 1) / BITS;
  static constexpr int T = WAVES * 64 * IPT;
  static constexpr int HW = D * R;
  union U {
    uint32_t hist[LCOPIES * (HW + 1)];
    struct P {
      uint32_t stage[T];
      uint32_t cnt[WAVES * R];
    } p;
  } u;
  uint32_t base[HW];     // segment-wide exclusive bucket starts, per digit
  uint32_t running[R];   // next free slot of each bucket in the current digit sweep
  uint32_t lbase[R + 1]; // tile-local bucket starts (+ tile size)
  uint32_t tot[R];       // tile bucket totals
  uint32_t scan[WAVES];
  uint32_t flag[kMaxDigits];
  uint32_t item;
};

// Splitters of a sorted segment: splitter p-1 = first key of cell p of P equal cells, all-ones
// for an empty cell (Sec. 1.1, footnote to Sec. 3.4.2).  Called after a workgroup barrier that
// follows the segment's last writes.
template <int THREADS>
__device__ __forceinline__ void seg_splitters(const SegDesc& dsc, uint32_t len) {
  if (!dsc.spl) return;
  __syncthreads();
  const uint32_t P = dsc.P, q = len / P, r = len % P;
  const gptr<uint32_t> spl = gmem(dsc.spl), out = gmem(dsc.dst);
  for (uint32_t p = threadIdx.x + 1; p < P; p += THREADS) {
    const uint64_t start = (uint64_t)p * q + (p < r ? p : r);
    spl[p - 1] = start < len ? out[start] : 0xFFFFFFFFu;
  }
}

// Tile rank of the keys k[] (wave-striped order) by the digit at `shift`: per-wave LDS counters,
// then one scan gives cnt[w][v] = tile-local start of wave w's run of bucket v, lbase (bucket
// starts) and tot (bucket totals).  SEG_RANK_ATOMIC ranks with lane-ordered LDS atomics
// (rank_slot), which the host selects only on a device that passed the lane-order check;
// SEG_RANK_BALLOT ranks with one ballot per digit bit (rank_ballot) and needs no ordering
// property of the LDS.
enum SegRank : int { SEG_RANK_ATOMIC = 0, SEG_RANK_BALLOT = 1 };

template <int BITS, int WAVES, int IPT, int LCOPIES, int RANK>
__device__ __forceinline__ void seg_rank_tile(SegSmem<BITS, WAVES, IPT, LCOPIES>& sm, const uint32_t (&k)[IPT],
                                              uint32_t (&r)[IPT], int shift) {
  constexpr int R = 1 << BITS, THREADS = WAVES * 64;
  const int tid = threadIdx.x, wid = tid >> 6;
  for (int j = tid; j < WAVES * R; j += THREADS) sm.u.p.cnt[j] = 0u;
  __syncthreads();
  uint32_t* cnt = sm.u.p.cnt + wid * R;
  if constexpr (RANK == SEG_RANK_ATOMIC) {
#pragma unroll
    for (int j = 0; j < IPT; ++j) r[j] = rank_slot(cnt, (k[j] >> shift) & (R - 1));
  } else {
#pragma unroll
    for (int j = 0; j < IPT; ++j) r[j] = rank_ballot<BITS>(cnt, (k[j] >> shift) & (R - 1));
  }
  tile_bucket_offsets<R, WAVES>(sm.u.p.cnt, sm.lbase, sm.scan);
  for (int b = tid; b < R; b += THREADS) sm.tot[b] = sm.lbase[b + 1] - sm.lbase[b];
  __syncthreads();
}

// A segment of len <= T keys sorted by the workgroup entirely in registers and LDS: per digit a
// rank, a constant-digit test and a reorder through LDS; one read and one write of every key
// (src == dst allowed: every key is in registers before the first write).  Then the splitters.
template <int BITS, int WAVES, int IPT, int LCOPIES, int RANK>
__device__ __forceinline__ void seg_sort_one_tile(SegSmem<BITS, WAVES, IPT, LCOPIES>& sm, const SegDesc& dsc,
                                                  uint32_t len) {
  using SM = SegSmem<BITS, WAVES, IPT, LCOPIES>;
  constexpr int R = SM::R, D = SM::D, T = SM::T, THREADS = WAVES * 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  uint32_t k[IPT], r[IPT];
  const uint32_t lb0 = (uint32_t)(wid * 64 * IPT + lane);
  const gptr<const uint32_t> in = gmem(dsc.src);
  const gptr<uint32_t> out = gmem(dsc.dst);
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint32_t idx = lb0 + j * 64;
    k[j] = idx < len ? in[idx] : 0xFFFFFFFFu;
  }
  const uint32_t nsent = (uint32_t)T - len;
#pragma unroll 1
  for (int d = 0; d < D; ++d) {
    const int shift = d * BITS;
    seg_rank_tile<BITS, WAVES, IPT, LCOPIES, RANK>(sm, k, r, shift);
    // constant digit over the segment's keys (sentinels sit in the largest bucket)
    if (tid == 0) sm.flag[0] = 0u;
    __syncthreads();
    const uint32_t vmax = (0xFFFFFFFFu >> shift) & (R - 1);
    for (int b = tid; b < R; b += THREADS)
      if (sm.tot[b] - ((uint32_t)b == vmax ? nsent : 0u) == len) sm.flag[0] = 1u;
    __syncthreads();
    if (sm.flag[0]) continue;  // uniform across the workgroup
    uint32_t* cnt = sm.u.p.cnt + wid * R;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const uint32_t v = (k[j] >> shift) & (R - 1);
      sm.u.p.stage[cnt[v] + r[j]] = k[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) k[j] = sm.u.p.stage[lb0 + j * 64];
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint32_t idx = lb0 + j * 64;
    if (idx < len) out[idx] = k[j];
  }
  seg_splitters<THREADS>(dsc, len);
}

// The single-array sort of a short array (n <= T) in one launch: one workgroup, seg_sort_one_tile.
template <int BITS, int WAVES, int IPT, int LCOPIES, int RANK>
__global__ __launch_bounds__(WAVES * 64) void k_sort_small(const uint32_t* src, uint32_t* dst, uint32_t n, uint32_t P,
                                                          uint32_t* spl) {
  __shared__ SegSmem<BITS, WAVES, IPT, LCOPIES> sm;
  SegDesc dsc;
  dsc.src = src;
  dsc.dst = dst;
  dsc.tmp = nullptr;
  dsc.spl = spl;
  dsc.n = n;
  dsc.P = P;
  dsc.pad[0] = dsc.pad[1] = 0u;
  seg_sort_one_tile<BITS, WAVES, IPT, LCOPIES, RANK>(sm, dsc, n);
}

// Persistent segmented sort over the descriptors order[lo..hi), longest first.  With
// item_hi == ~0u the range is that of the length classes [cls_lo, cls_hi] in the device-built
// work order (classes are stored longest first); otherwise it is [item_lo, item_hi).  Work items
// are taken from ctl->head[grp].
template <int BITS, int WAVES, int IPT, int LCOPIES, int RANK>
__global__ __launch_bounds__(WAVES * 64) void k_seg_sort(const SegDesc* __restrict__ order, uint32_t item_lo,
                                                        uint32_t item_hi, int cls_lo, int cls_hi, int grp,
                                                        SegCtl* __restrict__ ctl) {
  using SM = SegSmem<BITS, WAVES, IPT, LCOPIES>;
  constexpr int R = SM::R, D = SM::D, T = SM::T, HW = SM::HW, THREADS = WAVES * 64;
  constexpr int CS = HW + 1;
  __shared__ SM sm;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  uint32_t lo = item_lo, hi = item_hi;
  if (item_hi == ~0u) {
    lo = ctl->start[cls_hi];
    hi = ctl->start[cls_lo] + ctl->count[cls_lo];
  }

  while (true) {
    __syncthreads();
    if (tid == 0) sm.item = lo + add_agent(&ctl->head[grp], 1u);
    __syncthreads();
    const uint32_t item = sm.item;
    if (item >= hi) break;
    const SegDesc dsc = order[item];
    const uint32_t len = dsc.n;

    if (len <= (uint32_t)T) {
      seg_sort_one_tile<BITS, WAVES, IPT, LCOPIES, RANK>(sm, dsc, len);
      continue;
    }

    // ---------------- longer segment: histogram sweep, then one sweep per digit ----------------
    const gptr<const uint32_t> seg = gmem(dsc.src);
    for (int i = tid; i < LCOPIES * CS; i += THREADS) sm.u.hist[i] = 0u;
    __syncthreads();
    {
      uint32_t* hc = sm.u.hist + (tid % LCOPIES) * CS;
      auto count = [&](uint32_t key) {
#pragma unroll
        for (int d = 0; d < D; ++d) atomicAdd(&hc[d * R + ((key >> (d * BITS)) & (R - 1))], 1u);
      };
      uint32_t head = (uint32_t)(((16u - ((uintptr_t)seg & 15u)) & 15u) >> 2);
      if (head > len) head = len;
      if ((uint32_t)tid < head) count(seg[tid]);
      // 16-byte loads through a clang vector type (HIP's uint4 class has no copy from a global
      // reference)
      typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
      const gptr<const u32x4> v4 = reinterpret_cast<gptr<const u32x4>>(seg + head);
      const uint32_t nv = (len - head) >> 2;
      uint32_t i = tid;
      for (; i + 3 * THREADS < nv; i += 4 * THREADS) {
        const u32x4 x0 = v4[i], x1 = v4[i + THREADS], x2 = v4[i + 2 * THREADS], x3 = v4[i + 3 * THREADS];
        count(x0.x); count(x0.y); count(x0.z); count(x0.w);
        count(x1.x); count(x1.y); count(x1.z); count(x1.w);
        count(x2.x); count(x2.y); count(x2.z); count(x2.w);
        count(x3.x); count(x3.y); count(x3.z); count(x3.w);
      }
      for (; i < nv; i += THREADS) {
        const u32x4 x = v4[i];
        count(x.x); count(x.y); count(x.z); count(x.w);
      }
      for (uint32_t j = head + nv * 4 + tid; j < len; j += THREADS) count(seg[j]);
    }
    if (tid < kMaxDigits) sm.flag[tid] = 0u;
    __syncthreads();
    for (int j = tid; j < HW; j += THREADS) {
      uint32_t c = 0u;
#pragma unroll
      for (int cp = 0; cp < LCOPIES; ++cp) c += sm.u.hist[cp * CS + j];
      sm.base[j] = c;
      if (c == len) sm.flag[j / R] = 1u;  // constant digit
    }
#pragma unroll 1
    for (int d = 0; d < D; ++d) lds_exclusive_scan<R, THREADS>(sm.base + d * R, sm.scan);

    // Sweep buffers: the first sweep reads src; the sweeps alternate between dst and tmp so that the
    // last one writes dst.  In place (src == dst) the first sweep must write tmp, and an odd number
    // of sweeps then ends in tmp, which is copied back.
    uint32_t npass = 0;
    for (int d = 0; d < D; ++d) npass += sm.flag[d] ? 0u : 1u;
    const bool inplace = dsc.src == dsc.dst;
    const gptr<uint32_t> g_dst = gmem(dsc.dst), g_tmp = gmem(dsc.tmp);
    gptr<const uint32_t> src = seg;
    gptr<uint32_t> dst = (inplace || !(npass & 1u)) ? g_tmp : g_dst;
    gptr<uint32_t> other = (dst == g_tmp) ? g_dst : g_tmp;
    const uint32_t ntile = (len + T - 1) / T;
    const uint32_t lb0 = (uint32_t)(wid * 64 * IPT + lane);
#pragma unroll 1
    for (int d = 0; d < D; ++d) {
      if (sm.flag[d]) continue;  // uniform across the workgroup
      const int shift = d * BITS;
      for (int b = tid; b < R; b += THREADS) sm.running[b] = sm.base[d * R + b];
      // The tiles of a segment are swept in order by this one workgroup, so the next tile is
      // known: its loads are issued as soon as the current tile's keys are in LDS and complete
      // while the current tile is written out.
      uint32_t k[IPT];
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const uint32_t idx = lb0 + j * 64;
        k[j] = idx < len ? src[idx] : 0xFFFFFFFFu;
      }
#pragma unroll 1
      for (uint32_t t = 0; t < ntile; ++t) {
        const uint32_t tb = t * (uint32_t)T;
        uint32_t r[IPT];
        seg_rank_tile<BITS, WAVES, IPT, LCOPIES, RANK>(sm, k, r, shift);
        uint32_t* cnt = sm.u.p.cnt + wid * R;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          const uint32_t v = (k[j] >> shift) & (R - 1);
          sm.u.p.stage[cnt[v] + r[j]] = k[j];
        }
        if (t + 1 < ntile) {
#pragma unroll
          for (int j = 0; j < IPT; ++j) {
            const uint32_t idx = tb + (uint32_t)T + lb0 + j * 64;
            k[j] = idx < len ? src[idx] : 0xFFFFFFFFu;
          }
        }
        __syncthreads();
        const uint32_t nvalid = (len - tb) < (uint32_t)T ? (len - tb) : (uint32_t)T;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
          const uint32_t i = (uint32_t)(j * THREADS + tid);
          if (i < nvalid) {
            const uint32_t key = sm.u.p.stage[i];
            const uint32_t v = (key >> shift) & (R - 1);
            dst[sm.running[v] + i - sm.lbase[v]] = key;
          }
        }
        __syncthreads();
        for (int b = tid; b < R; b += THREADS) sm.running[b] += sm.tot[b];
      }
      src = dst;
      gptr<uint32_t> nxt = other;
      other = dst;
      dst = nxt;
      __syncthreads();  // this sweep's writes are complete before the next sweep reads them
    }
    if (src != g_dst) {  // no sweep ran (copy) or, in place, an odd number ended in tmp
      for (uint32_t i = tid; i < len; i += THREADS) g_dst[i] = src[i];
    }
    __syncthreads();
    seg_splitters<THREADS>(dsc, len);
  }

  // last workgroup out resets this group's counters for the next call
  if (tid == 0) {
    __threadfence();
    if (add_agent(&ctl->done2[grp], 1u) == gridDim.x - 1) {
      st_agent(&ctl->head[grp], 0u);
      st_agent(&ctl->done2[grp], 0u);
    }
  }
}

// Clears the per-call part of the control block after every group kernel has run.
__global__ void k_seg_reset(SegCtl* __restrict__ ctl) {
  const int t = threadIdx.x;
  if (t < kSegBuckets) {
    ctl->count[t] = 0u;
    ctl->start[t] = 0u;
    ctl->cursor[t] = 0u;
  }
  if (t == 0) {
    ctl->nwork = 0u;
    ctl->bad = 0u;
    ctl->long_cursor = 0ull;
  }
  if (t < 4) ctl->long_ctr[t] = 0u;
}

}  // namespace aps
