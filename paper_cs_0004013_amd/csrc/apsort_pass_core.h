// One tile of one digit pass of the LSD radix sort (Sec. 3.2 partial sort + distribution for one
// digit, Sec. 3.3.1 digit order), shared by the single-array pass (k_pass) and the device-wide pass
// over the long segments of a batched sort (k_seg_long_pass).  Templates only.
//
// A tile is T = WAVES*64*IPT keys, taken wave-striped (key j of lane l of wave w sits at
// w*64*IPT + j*64 + l), which is memory order in (w, j, l) order, so ranking sub-step j of every
// wave in order is stable.  Order of work in a tile: load; rank; publish the tile's bucket counts;
// tile-local scan; reorder the keys in LDS; decoupled look-back for the global bucket starts (the
// per-cell-per-bucket totals that Sec. 3.2 chose not to communicate, so placement is exact);
// write the reordered keys out, runs of one bucket to consecutive addresses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apsort_device.h"

namespace aps {

// Rank primitives of the digit pass.
enum RankKind : int {
  RANK_ATOMIC = 0,  // LDS add-with-return on per-wave counters; relies on the LDS servicing the
                    // conflicting lanes of one instruction in ascending lane order (checked on the
                    // device by k_lane_order_probe before this kind is used)
  RANK_MATCH = 1    // per-wave LDS lane masks (OR, read, clear) + leader update; order-agnostic
};

// The LDS arrays of a digit pass.  The kernel declares them as separate __shared__ arrays and
// passes this view: the compiler then places the 128 KiB stage first and aligns each array on its
// own, and the pass measured 3.5% faster than with the same arrays as members of one __shared__
// struct (same instructions, other LDS offsets).
template <int BITS, int WAVES, int IPT, int RANK, bool KV>
struct PassSmem {
  static constexpr int R = 1 << BITS;
  static constexpr int T = WAVES * 64 * IPT;
  uint32_t* cnt;    // [WAVES * R] per-wave bucket counters, then per-wave run starts
  uint32_t* lbase;  // [R + 1] tile-local bucket starts (+ tile size)
  uint32_t* delta;  // [R] global start minus tile-local start, per bucket
  uint32_t* stage;  // [T] keys in tile-sorted order
  uint32_t* vstage; // [T] their values (pairs only)
  uint32_t* scan;   // [WAVES]
  uint64_t* bins;   // [WAVES * R] per-wave bucket lane masks (mask rank only)
};

// Declares the LDS arrays of a digit pass in the calling kernel and the view `name` of them.
#define AP_PASS_SMEM(name, BITS, WAVES, IPT, RANK, KV)                                              \
  __shared__ uint32_t name##_cnt[(WAVES) * (1 << (BITS))];                                          \
  __shared__ uint32_t name##_lbase[(1 << (BITS)) + 1];                                              \
  __shared__ uint32_t name##_delta[1 << (BITS)];                                                    \
  __shared__ uint32_t name##_stage[(WAVES) * 64 * (IPT)];                                           \
  __shared__ uint32_t name##_vstage[(KV) ? (WAVES) * 64 * (IPT) : 1];                               \
  __shared__ uint32_t name##_scan[WAVES];                                                           \
  __shared__ uint64_t name##_bins[(RANK) == RANK_MATCH ? (WAVES) * (1 << (BITS)) : 1];              \
  const PassSmem<BITS, WAVES, IPT, RANK, KV> name{name##_cnt,   name##_lbase, name##_delta, name##_stage, \
                                                  name##_vstage, name##_scan, name##_bins}

// Clears the counters of the next tile (every thread takes part; a barrier must follow).
template <int BITS, int WAVES, int IPT, int RANK, bool KV>
__device__ __forceinline__ void pass_clear(const PassSmem<BITS, WAVES, IPT, RANK, KV>& sm) {
  constexpr int R = 1 << BITS, THREADS = WAVES * 64;
  for (int j = threadIdx.x; j < WAVES * R; j += THREADS) sm.cnt[j] = 0u;
  if constexpr (RANK == RANK_MATCH)
    for (int j = threadIdx.x; j < WAVES * R; j += THREADS) sm.bins[j] = 0ull;
}

// Debug modes of the digit pass, compiled only into the k_pass_dbg instantiations (the default
// kernels carry none of this code).
//   PASS_DBG_PERTURB: seeded delays of up to ~10 us at the tile claim and before the aggregate,
//     the reorder, the inclusive prefix and the scatter, so that tiles publish and finish in an
//     order the normal timing seldom produces (a stress of the look-back and the claim order).
//   PASS_DBG_TRACE: wall-clock timestamps (s_memrealtime, 100 MHz) at the tile's phase boundaries,
//     written by thread 0 as kPassTraceWords words per tile at trace[(pass * ntiles + tile) * 8];
//     the trace build adds a barrier after the rank and after the reorder, and waits for the
//     scatter's stores, so that each phase ends for the whole workgroup at its timestamp.
enum PassDebug : int { PASS_DBG_NONE = 0, PASS_DBG_PERTURB = 1, PASS_DBG_TRACE = 2 };
constexpr int kPassTraceWords = 8;  // claim, rank, scan, reorder, look-back, scatter, 2 spare
struct PassDebugArgs {
  uint64_t seed;                    // perturbation seed
  unsigned long long* trace;        // trace records (NULL: none)
  uint64_t trace_records;           // capacity in records of kPassTraceWords words
  uint32_t record0;                 // record index of tile 0 of this pass (pass * ntiles)
  uint32_t pad;
};

__device__ __forceinline__ uint64_t dbg_mix(uint64_t z) {  // SplitMix64 finaliser
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// A seeded delay, the same for every thread of the workgroup: no delay on half of the draws,
// otherwise up to three sleeps of 8128 cycles plus up to 4032 (about 0 - 12 us at 2.4 GHz).
__device__ __forceinline__ void dbg_delay(const PassDebugArgs& dbg, uint32_t tile, int shift, int point) {
  const uint64_t h = dbg_mix(dbg.seed ^ ((uint64_t)tile << 16) ^ ((uint64_t)shift << 8) ^ (uint64_t)point);
  if (h & 1u) return;
  for (uint32_t i = 0; i < (uint32_t)((h >> 1) & 3u); ++i) __builtin_amdgcn_s_sleep(127);
  for (uint32_t i = 0; i < (uint32_t)((h >> 3) & 63u); ++i) __builtin_amdgcn_s_sleep(1);
}
__device__ __forceinline__ void dbg_stamp(const PassDebugArgs& dbg, uint32_t tile, int word) {
  if (threadIdx.x == 0 && dbg.trace && (uint64_t)dbg.record0 + tile < dbg.trace_records)
    dbg.trace[((uint64_t)dbg.record0 + tile) * kPassTraceWords + word] = __builtin_amdgcn_s_memrealtime();
}

// The tile `tile` of the array src[0..n) (keys past n are all-ones sentinels: largest digit, last
// in order, never written) for the digit at `shift`.  g_base[v] = number of keys of the whole array
// with a smaller digit; status = look-back words of this array's tiles (R per tile, 2-bit state +
// 30-bit count, zero before the pass).  The counters must have been cleared (pass_clear + barrier).
// tid = threadIdx.x (a persistent caller passes it through an opaque copy, so that the addresses
// derived from it are not hoisted out of its loop and kept in registers for every tile).
// NT_STORE (keys only): scatter with the non-temporal hint, else with plain stores.  NT_LOAD_KV
// (pairs only): full-tile loads of keys and values with the non-temporal hint.  Template
// parameters: with a run-time flag the compiler merges the two accesses into one plain access.
template <int BITS, int WAVES, int IPT, int RANK, int LB_WIN, bool KV, int DBG = PASS_DBG_NONE, bool NT_STORE = true,
          bool NT_LOAD_KV = false>
__device__ __forceinline__ void pass_tile(const PassSmem<BITS, WAVES, IPT, RANK, KV>& sm, const uint32_t* __restrict__ src,
                                          uint32_t* __restrict__ dst, const uint32_t* __restrict__ vsrc,
                                          uint32_t* __restrict__ vdst, uint32_t n, uint32_t tile, int shift,
                                          const uint32_t* __restrict__ g_base, uint32_t* __restrict__ status,
                                          int tid, const PassDebugArgs* dbg = nullptr) {
  constexpr int R = 1 << BITS;
  constexpr int THREADS = WAVES * 64;
  constexpr int T = THREADS * IPT;
  constexpr int BPT = (R + THREADS - 1) / THREADS;
  const int lane = tid & 63, wid = tid >> 6;
  const uint32_t tbase = tile * (uint32_t)T;
  // global views: the long-segment pass reads these pointers from descriptors
  const gptr<const uint32_t> gsrc = gmem(src), gvsrc = gmem(vsrc);
  const gptr<uint32_t> gdst = gmem(dst), gvdst = gmem(vdst);

  // ---- load ----
  uint32_t k[IPT];
  uint32_t val[KV ? IPT : 1];
  const uint32_t wbase = tbase + (uint32_t)(wid * 64 * IPT + lane);
  // Every key is read once and written once per pass: for keys alone the loads carry the
  // non-temporal hint (3-7% faster per sort), and so do the stores unless the caller asks for
  // plain ones (NT_STORE false: a pass whose output the next pass reads, on arrays large enough
  // that the merged run-boundary lines and the cache hits of the next pass pay).  With values beside the keys (two streams each way) the hint on
  // stores made passes ~30% slower, so pairs store plainly, and load with the hint only where the
  // caller asks (NT_LOAD_KV: arrays whose keys and values just fit the last-level cache).
  if (tbase + (uint32_t)T <= n) {
    if constexpr (KV && NT_LOAD_KV) {
#pragma unroll
      for (int j = 0; j < IPT; ++j) k[j] = __builtin_nontemporal_load(&gsrc[wbase + j * 64]);
#pragma unroll
      for (int j = 0; j < IPT; ++j) val[j] = __builtin_nontemporal_load(&gvsrc[wbase + j * 64]);
    } else if constexpr (KV) {
#pragma unroll
      for (int j = 0; j < IPT; ++j) k[j] = gsrc[wbase + j * 64];
#pragma unroll
      for (int j = 0; j < IPT; ++j) val[j] = gvsrc[wbase + j * 64];
    } else {
#pragma unroll
      for (int j = 0; j < IPT; ++j) k[j] = __builtin_nontemporal_load(&gsrc[wbase + j * 64]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const uint32_t idx = wbase + j * 64;
      k[j] = idx < n ? gsrc[idx] : 0xFFFFFFFFu;
      if constexpr (KV) val[j] = idx < n ? gvsrc[idx] : 0u;
    }
  }

  // ---- A4: stable rank within the wave's keys ----
  uint32_t r[IPT];
  uint32_t* cnt = sm.cnt + wid * R;
  if constexpr (RANK == RANK_ATOMIC) {
    // lane-ordered LDS atomics (rank_slot), one add of 64 for a slot of one digit
#pragma unroll
    for (int j = 0; j < IPT; ++j) r[j] = rank_slot(cnt, (k[j] >> shift) & (R - 1));
  } else {
    // Every lane ORs its lane bit into its bucket's 64-bit word, reads the word back (the lanes of
    // this sub-step sharing the bucket) and clears it; the lowest such lane updates the counter.
    uint64_t* bins = sm.bins + wid * R;
    const uint64_t mybit = 1ull << lane;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const uint32_t v = (k[j] >> shift) & (R - 1);
      // Each step needs every lane of the wave to have finished the previous one: a wave's LDS
      // instructions run for all its lanes before the next starts.  The wave barriers (no
      // instruction, only a scheduling fence) state that order where lanes do not run together.
      __hip_atomic_fetch_or(&bins[v], mybit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      __builtin_amdgcn_wave_barrier();
      const uint64_t m = __hip_atomic_load(&bins[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      __builtin_amdgcn_wave_barrier();
      __hip_atomic_store(&bins[v], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      const uint32_t peers = lanes_below(m);
      const uint32_t c = cnt[v];
      __builtin_amdgcn_wave_barrier();
      r[j] = c + peers;
      if (peers == 0u) cnt[v] = c + (uint32_t)__popcll(m);
      __builtin_amdgcn_wave_barrier();
    }
  }

  // ---- tile-local run starts (one scan over bucket-major, wave-minor counts); publish the
  //      tile's bucket counts for the look-back of later tiles ----
  if constexpr (DBG == PASS_DBG_TRACE) {
    __syncthreads();
    dbg_stamp(*dbg, tile, 1);
  }
  if constexpr (DBG == PASS_DBG_PERTURB) dbg_delay(*dbg, tile, shift, 1);
  tile_bucket_offsets<R, WAVES>(sm.cnt, sm.lbase, sm.scan);
  if constexpr (DBG == PASS_DBG_TRACE) dbg_stamp(*dbg, tile, 2);
  uint32_t tot[BPT];
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int b = tid + i * THREADS;
    tot[i] = 0u;
    if (b < R) {
      tot[i] = sm.lbase[b + 1] - sm.lbase[b];
      if (tile == 0u) st_agent(status + b, kFlagPrefix | (g_base[b] + tot[i]));
      else st_agent(status + (size_t)tile * R + b, kFlagAgg | tot[i]);
    }
  }

  if constexpr (DBG == PASS_DBG_PERTURB) dbg_delay(*dbg, tile, shift, 2);
  // ---- A5 (first half): reorder the tile in LDS; independent of the global offsets ----
  uint32_t* cnt_w = sm.cnt + wid * R;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint32_t v = (k[j] >> shift) & (R - 1);
    sm.stage[cnt_w[v] + r[j]] = k[j];
    if constexpr (KV) sm.vstage[cnt_w[v] + r[j]] = val[j];
  }

  if constexpr (DBG == PASS_DBG_TRACE) {
    __syncthreads();
    dbg_stamp(*dbg, tile, 3);
  }
  if constexpr (DBG == PASS_DBG_PERTURB) dbg_delay(*dbg, tile, shift, 3);
  // ---- A3: decoupled look-back for each bucket's global start ----
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int b = tid + i * THREADS;
    if (b < R) {
      uint32_t excl;
      if (tile == 0u) {
        excl = g_base[b];
      } else {
        // Sum the published counts of the preceding tiles, newest first, until one of them has
        // published its inclusive prefix; LB_WIN status words (one per preceding tile) are
        // fetched per round trip.
        excl = 0u;
        int p = (int)tile - 1;
        while (true) {
          uint32_t sv[LB_WIN];
#pragma unroll
          for (int q = 0; q < LB_WIN; ++q) sv[q] = (p - q >= 0) ? ld_agent(status + (size_t)(p - q) * R + b) : 0u;
          int used = 0;
          bool done = false;
#pragma unroll
          for (int q = 0; q < LB_WIN; ++q) {
            if (!done && used == q) {
              const uint32_t f = sv[q] & kFlagMask;
              if (f != 0u) {
                excl += sv[q] & kValueMask;
                ++used;
                done = (f == kFlagPrefix);
              }
            }
          }
          if (done) break;
          p -= used;
          if (used == 0) __builtin_amdgcn_s_sleep(1);
        }
        if constexpr (DBG == PASS_DBG_PERTURB) dbg_delay(*dbg, tile, shift, 4);
        st_agent(status + (size_t)tile * R + b, kFlagPrefix | (excl + tot[i]));
      }
      sm.delta[b] = excl - sm.lbase[b];
    }
  }
  __syncthreads();
  if constexpr (DBG == PASS_DBG_TRACE) dbg_stamp(*dbg, tile, 4);
  if constexpr (DBG == PASS_DBG_PERTURB) dbg_delay(*dbg, tile, shift, 5);

  // ---- A5 (second half): coalesced scatter; runs of one bucket go to consecutive addresses ----
  const uint32_t nvalid = (n - tbase) < (uint32_t)T ? (n - tbase) : (uint32_t)T;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint32_t i = (uint32_t)(j * THREADS + tid);
    if (i < nvalid) {
      const uint32_t key = sm.stage[i];
      const uint32_t v = (key >> shift) & (R - 1);
      if constexpr (KV) {
        gdst[sm.delta[v] + i] = key;
        gvdst[sm.delta[v] + i] = sm.vstage[i];
      } else if constexpr (NT_STORE) {
        __builtin_nontemporal_store(key, &gdst[sm.delta[v] + i]);
      } else {
        gdst[sm.delta[v] + i] = key;
      }
    }
  }
  if constexpr (DBG == PASS_DBG_TRACE) {
    __builtin_amdgcn_s_waitcnt(0);  // every counter zero: this thread's stores have completed
    __syncthreads();
    dbg_stamp(*dbg, tile, 5);
  }
}

}  // namespace aps
