// Device-side helpers shared by every kernel of libapsort.so: plan words, look-back status word
// format, memory-scope helpers, wave primitives and an LDS scan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aps {

// ---- pass plan, written by the last workgroup of k_hist_plan, read by k_pass / k_finalize ----
constexpr int kMaxDigits = 8;  // digit width >= 4 bits
enum PlanWord : int {
  PL_RUN = 0,              // [kMaxDigits] 1 when pass d runs
  PL_SRC = 8,              // [kMaxDigits] buffer selector read by pass d
  PL_DST = 16,             // [kMaxDigits] buffer selector written by pass d
  PL_NPASS = 24,           // number of passes that run
  PL_FINAL = 25,           // selector of the buffer holding the sorted keys after the last pass
  PL_COPY = 26,            // 1 when k_finalize must copy PL_FINAL into the output
  PL_WORDS = 32
};
enum BufSel : uint32_t { SEL_IN = 0, SEL_OUT = 1, SEL_TMP = 2 };

// ---- look-back status word: 2-bit state | 30-bit count ----
constexpr uint32_t kFlagMask = 3u << 30;
constexpr uint32_t kFlagAgg = 1u << 30;     // tile's own bucket count is published
constexpr uint32_t kFlagPrefix = 2u << 30;  // inclusive prefix through this tile is published
constexpr uint32_t kValueMask = (1u << 30) - 1;

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_agent(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent_u64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Global-memory view of a pointer.  A pointer that a kernel reads from memory (a descriptor field)
// is generic to the compiler, which then accesses it with flat instructions.  A flat access counts
// against the LDS wait counter as well as the vector-memory one, so every LDS wait of a rank or a
// scatter would also wait for all global loads and stores in flight.  Pointers that are kernel
// arguments are known to be global already.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}

// Number of set bits of m in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Mask of the lanes of the (fully active) wave whose BITS-bit value equals the caller's.
// One ballot per bit: keep the lanes that agree with this lane on every bit.
template <int BITS>
__device__ __forceinline__ uint64_t match_any(uint32_t v) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const bool bit = (v >> b) & 1u;
    const uint64_t bal = __builtin_amdgcn_ballot_w64(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

// Stable rank of this lane's digit v among the wave's keys ranked so far, against the wave's own
// LDS counters cnt (one word per digit), with no assumption on the order in which the LDS serves
// conflicting lanes: the lanes sharing v are found with match_any, a lane's rank is the counter
// plus the number of those lanes below it, and the lowest of them advances the counter.  Every
// lane of the wave must be active.  A wave's LDS instructions run in program order, so every
// lane's read of the counter completes before the leaders write it.
template <int BITS>
__device__ __forceinline__ uint32_t rank_ballot(uint32_t* cnt, uint32_t v) {
  const uint64_t m = match_any<BITS>(v);
  const uint32_t peers = lanes_below(m);
  const uint32_t c = cnt[v];
  __builtin_amdgcn_wave_barrier();
  if (peers == 0u) cnt[v] = c + (uint32_t)__popcll(m);
  __builtin_amdgcn_wave_barrier();
  return c + peers;
}

// Stable rank of this lane's digit v among the wave's keys ranked so far, against the wave's own
// LDS counters cnt (one word per digit).  LDS executes one wave's instructions in order and
// services the conflicting lanes of one instruction in lane order, so the value an atomic
// increment returns is the number of this wave's earlier keys (earlier instructions, then lower
// lanes) with the same digit.  Lanes sharing a digit queue on one LDS word, lane by lane; when
// every lane holds lane 0's digit (runs of equal keys, as earlier passes bring them together),
// lane 0 adds 64 once and lane l's rank is the old count + l, the same result.  (Ranking slots
// with a few shared digits by digit leaders measured slower than the atomics on every key set
// tried.)
__device__ __forceinline__ uint32_t rank_slot(uint32_t* cnt, uint32_t v) {
  const uint32_t v0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
  if (__builtin_amdgcn_ballot_w64(v == v0) == ~0ull) {
    uint32_t old = 0u;
    if ((threadIdx.x & 63u) == 0u)
      old = __hip_atomic_fetch_add(&cnt[v0], 64u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return (uint32_t)__builtin_amdgcn_readlane((int)old, 0) + (threadIdx.x & 63u);
  }
  return __hip_atomic_fetch_add(&cnt[v], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// In-place exclusive scan of a[0..N) in LDS by the whole workgroup; returns the total.
// scratch needs THREADS/64 words.  Starts and ends with a workgroup barrier.
template <int N, int THREADS>
__device__ __forceinline__ uint32_t lds_exclusive_scan(uint32_t* a, uint32_t* scratch) {
  constexpr int C = (N + THREADS - 1) / THREADS;
  constexpr int W = THREADS / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  uint32_t local[C];
  uint32_t sum = 0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int idx = tid * C + c;
    local[c] = idx < N ? a[idx] : 0u;
    sum += local[c];
  }
  uint32_t x = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) scratch[wid] = x;
  __syncthreads();
  uint32_t wpre = 0, total = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t s = scratch[w];
    wpre += (w < wid) ? s : 0u;
    total += s;
  }
  uint32_t run = wpre + x - sum;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int idx = tid * C + c;
    if (idx < N) a[idx] = run;
    run += local[c];
  }
  __syncthreads();
  return total;
}

// Tile bucket offsets from per-wave bucket counts, with one block-wide scan.
// On entry cnt[w*R + b] = number of keys of wave w in bucket b.  On exit cnt[w*R + b] = tile-local
// start of wave w's run of bucket b, i.e. the exclusive prefix over (bucket, wave) in bucket-major
// order, so runs of one bucket follow wave order (stable); lbase[b] = start of bucket b and
// lbase[R] = number of keys in the tile.  scratch needs WAVES words.  Starts and ends with a
// workgroup barrier.
template <int R, int WAVES>
__device__ __forceinline__ void tile_bucket_offsets(uint32_t* cnt, uint32_t* lbase, uint32_t* scratch) {
  constexpr int THREADS = WAVES * 64, N = R * WAVES, E = (N + THREADS - 1) / THREADS;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  uint32_t v[E];
  uint32_t sum = 0u;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int f = tid * E + e;
    v[e] = f < N ? cnt[(f % WAVES) * R + f / WAVES] : 0u;
    sum += v[e];
  }
  uint32_t x = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) scratch[wid] = x;
  __syncthreads();
  uint32_t run = x - sum;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) run += (w < wid) ? scratch[w] : 0u;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int f = tid * E + e;
    if (f < N) {
      const int b = f / WAVES, w = f % WAVES;
      cnt[w * R + b] = run;
      if (w == 0) lbase[b] = run;
    }
    run += v[e];
  }
  if (tid == THREADS - 1) lbase[R] = run;
  __syncthreads();
}

}  // namespace aps
