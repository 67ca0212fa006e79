// Device kernels of the radix sort (gfx950, wave64).  Included by the host translation units;
// everything here is header-only templates so that each entry point instantiates exactly the
// configurations it launches.
//
// Step map (Weaver & Lynes, "Sorting Integers on the AP1000"):
//   k_hist_plan   Sec. 3.2 first loop of bucket(): bucket counts of every digit in one read of the
//                 keys; then cumulative totals (exclusive scan, Sec. 3.2 and the scan-before-sum
//                 ordering of Sec. 4.4) and the pass plan (constant digits are skipped, the exact
//                 form of the 30-bit shortcut of Sec. 4.5).
//   k_pass        Sec. 3.2 partial sort + distribution for one digit of the LSD sort (Sec. 3.3.1):
//                 tile-local stable ranking, a single-pass scan of per-tile bucket counts with
//                 decoupled look-back (the per-cell-per-bucket totals that Sec. 3.2 chose not to
//                 communicate, so placement here is exact), and a scatter staged through LDS; the
//                 per-tile work is pass_tile (apsort_pass_core.h).
//   k_finalize    Sec. 1.1 output contract: copy when no pass wrote the output, and the P-1
//                 splitters (first key of each cell, footnote to Sec. 3.4.2 for uneven counts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apsort_device.h"
#include "apsort_pass_core.h"

namespace aps {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

// ------------------------------------------------------------------------------------------------
// A1 + A2: bucket counts of all digits in one read, then (last workgroup) constant-digit flags,
// exclusive scans and the pass plan.
//   g_hist   ncopies * D*R counters, zero on entry, left zero on exit (the last workgroup clears
//            them); workgroup g adds into copy g % ncopies so that fewer workgroups contend for
//            one counter
//   done     workgroup-completion counter, zero on entry and on exit
//   zero_ptr/zero_vec4  scan state of the passes (tile counters + status words), cleared here
//   out_hist optional copy of the final counts (inspection entry point)
//   first_digit  lowest digit the plan sorts on (0 for a full sort)
// Inside a workgroup, with 8-bit digits and 1024 threads (1024 counters), every lane position l
// of the wave owns a private copy of the counters as 16-bit halves: bucket B is the half B & 1 of
// LDS word (B / 2) * 64 + l, so the 64 lanes of one atomic add always hit 64 different banks
// (random digits would otherwise collide 4-5 fold per bank).  The 16 waves share the copies,
// hence the adds stay atomic; a copy counts the keys of 16 threads, at most
// 16 * (4 * kHistMaxVecPerThread + 2) < 2^16, which the host guarantees through the grid size.
// Other widths use LCOPIES full-word copies, lane l using copy l % LCOPIES, HW+1 words apart.
// ------------------------------------------------------------------------------------------------
constexpr uint32_t kHistMaxVecPerThread = 1023;  // 4-key vectors counted by one thread, at most
constexpr int kHistMaxCopies = 32;  // global copies of the counts (spreads the workgroups' atomic adds)
template <int BITS, int THREADS, int LCOPIES>
__global__ __launch_bounds__(THREADS) void k_hist_plan(
    const uint32_t* __restrict__ keys, uint32_t n, uint32_t* __restrict__ g_hist,
    uint32_t* __restrict__ g_base, uint32_t* __restrict__ plan, uint32_t* __restrict__ done,
    uint4* __restrict__ zero_ptr, uint32_t zero_vec4, int inplace, uint32_t* __restrict__ out_hist,
    uint32_t ncopies, int first_digit) {
  constexpr int R = 1 << BITS;
  constexpr int D = (32 + BITS - 1) / BITS;
  constexpr int HW = D * R;
  constexpr int CS = HW + 1;  // copy stride
  constexpr bool LANE_PRIV = (HW == 1024 && THREADS == 1024);
  // a lane copy counts the keys of THREADS / 64 threads: at most 4 per vector plus one head and
  // one tail key each
  static_assert(!LANE_PRIV || (THREADS / 64) * (4 * kHistMaxVecPerThread + 2) < 65536u,
                "16-bit lane counters would overflow");
  constexpr int HWORDS = LANE_PRIV ? (HW / 2) * 64 : LCOPIES * CS;
  __shared__ uint32_t h[HWORDS];
  __shared__ uint32_t s_const[kMaxDigits];
  __shared__ uint32_t s_scan[THREADS / 64];
  __shared__ int s_last;

  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < (uint32_t)HWORDS; i += THREADS) h[i] = 0u;
  const uint32_t gtid = blockIdx.x * THREADS + tid, gstride = gridDim.x * THREADS;
  for (uint32_t i = gtid; i < zero_vec4; i += gstride) zero_ptr[i] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();

  uint32_t* __restrict__ hc = LANE_PRIV ? h + (tid & 63u) : h + (tid % LCOPIES) * CS;
  auto count = [&](uint32_t k) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const uint32_t b = (uint32_t)(d * R) + ((k >> (d * BITS)) & (R - 1));
      if constexpr (LANE_PRIV) atomicAdd(&hc[(b >> 1) * 64u], 1u << ((b & 1u) * 16u));
      else atomicAdd(&hc[b], 1u);
    }
  };
  uint32_t head = (uint32_t)(((16u - ((uintptr_t)keys & 15u)) & 15u) >> 2);
  if (head > n) head = n;
  if (gtid < head) count(keys[gtid]);
  const uint4* __restrict__ v = reinterpret_cast<const uint4*>(keys + head);
  const uint32_t nv = (n - head) >> 2;
  uint32_t i = gtid;
  if (i + 3 * gstride < nv) {
    // Software pipelined over two register sets: the next four vectors are in flight while the
    // current four are counted.  rounds = number of r with i + 4*gstride*r + 3*gstride < nv.  The
    // loop has a fixed trip count and no exit between a load and its use (otherwise the compiler
    // sinks the loads below the counting); the last round of an even count re-reads the vectors
    // just loaded (cache hits) instead of branching around the load.
    const uint32_t step = 4 * gstride;
    const uint32_t rounds = (nv - 3 * gstride - i + step - 1) / step;
    auto load4 = [&](uint32_t r, uint4* q) {
      const uint32_t at = i + r * step;
      q[0] = v[at];
      q[1] = v[at + gstride];
      q[2] = v[at + 2 * gstride];
      q[3] = v[at + 3 * gstride];
    };
    auto count4 = [&](const uint4* q) {
#pragma unroll
      for (int u = 0; u < 4; ++u) { count(q[u].x); count(q[u].y); count(q[u].z); count(q[u].w); }
    };
    uint4 qa[4], qb[4];
    load4(0, qa);
    uint32_t r = 0;
    for (; r + 2 <= rounds; r += 2) {  // qa holds round r
      load4(r + 1, qb);
      count4(qa);
      load4(r + 2 < rounds ? r + 2 : r + 1, qa);
      count4(qb);
    }
    if (r < rounds) count4(qa);  // odd count: qa holds the last round
    i += rounds * step;
  }
  for (; i < nv; i += gstride) {
    const uint4 a = v[i];
    count(a.x); count(a.y); count(a.z); count(a.w);
  }
  for (uint32_t j = head + nv * 4 + gtid; j < n; j += gstride) count(keys[j]);
  __syncthreads();
  uint32_t* __restrict__ mine = g_hist + (size_t)(blockIdx.x % ncopies) * HW;
  for (uint32_t j = tid; j < HW; j += THREADS) {
    uint32_t c = 0u;
    if constexpr (LANE_PRIV) {
      // lane copies read in a rotated order: the 64 lanes of a read hit 64 different banks
      const uint32_t row = (j >> 1) * 64u, sh = (j & 1u) * 16u;
#pragma unroll 16
      for (uint32_t q = 0; q < 64u; ++q) c += (h[row + ((q + j) & 63u)] >> sh) & 0xFFFFu;
    } else {
#pragma unroll
      for (int cp = 0; cp < LCOPIES; ++cp) c += h[cp * CS + j];
    }
    if (c) add_agent(&mine[j], c);
  }
  // Last-workgroup-done: the barrier makes every thread's adds complete before thread 0's
  // release fence and completion count; the last workgroup's acquire fence pairs with those
  // fences.  One thread per workgroup fences (a device-scope fence writes back and invalidates
  // the L2, so it is kept off the other threads).
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    s_last = (add_agent(done, 1u) == gridDim.x - 1);
    if (s_last) __threadfence();
  }
  __syncthreads();
  if (!s_last) return;

  // ---- last workgroup: every count is in g_hist ----
  if (tid < kMaxDigits) s_const[tid] = 0u;
  __syncthreads();
  const uint32_t used = gridDim.x < ncopies ? gridDim.x : ncopies;
  for (uint32_t j = tid; j < HW; j += THREADS) {
    // every copy's count is loaded before any is summed: one round trip to memory, not one per
    // group of copies (the loads cross the XCDs' caches)
    uint32_t c = 0u;
    for (uint32_t cp0 = 0; cp0 < used; cp0 += kHistMaxCopies) {
      uint32_t part[kHistMaxCopies];
#pragma unroll
      for (int q = 0; q < kHistMaxCopies; ++q)
        part[q] = (cp0 + q < used) ? ld_agent(&g_hist[(size_t)(cp0 + q) * HW + j]) : 0u;
#pragma unroll
      for (int q = 0; q < kHistMaxCopies; ++q) c += part[q];
    }
    for (uint32_t cp = 0; cp < used; ++cp) g_hist[(size_t)cp * HW + j] = 0u;
    h[j] = c;
    if (out_hist) out_hist[j] = c;
    if (c == n) s_const[j / R] = 1u;  // one bucket holds every key: the digit is constant
  }
  if constexpr (HW == THREADS && R % 64 == 0) {
    // one counter per thread: every digit's exclusive scan at once (a wave scan, then the sums of
    // the digit's earlier waves), two barriers instead of three per digit
    __syncthreads();
    const uint32_t lane = tid & 63u, wid = tid >> 6;
    const uint32_t x0 = h[tid];
    uint32_t x = x0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= (uint32_t)off) x += y;
    }
    if (lane == 63u) s_scan[wid] = x;
    __syncthreads();
    constexpr uint32_t WPD = R / 64;  // waves per digit
    uint32_t pre = 0u;
    for (uint32_t w = wid / WPD * WPD; w < wid; ++w) pre += s_scan[w];
    g_base[tid] = pre + x - x0;
  } else {
#pragma unroll 1
    for (int d = 0; d < D; ++d) {
      lds_exclusive_scan<R, THREADS>(h + d * R, s_scan);
      for (uint32_t j = tid; j < R; j += THREADS) g_base[d * R + j] = h[d * R + j];
    }
  }
  if (tid == 0) {
    // Digits below first_digit are not sorted on here (the bucketing variant leaves them to the
    // local sorts of its buckets).
    uint32_t npass = 0;
    for (int d = first_digit; d < D; ++d) npass += s_const[d] ? 0u : 1u;
    // Ping-pong so that the last pass that runs writes the output: with an odd number of passes
    // the first one writes the output, with an even number it writes the scratch buffer.  In
    // place (in == out) the first pass must not write the input, so it always writes scratch.
    const uint32_t first_dst = inplace ? (uint32_t)SEL_TMP : ((npass & 1u) ? (uint32_t)SEL_OUT : (uint32_t)SEL_TMP);
    uint32_t cur = SEL_IN;
    for (int d = 0; d < kMaxDigits; ++d) {
      const uint32_t run = (d >= first_digit && d < D && !s_const[d]) ? 1u : 0u;
      plan[PL_RUN + d] = run;
      plan[PL_SRC + d] = cur;
      uint32_t nxt = cur;
      if (run) nxt = (cur == SEL_IN) ? first_dst : (cur == SEL_OUT ? (uint32_t)SEL_TMP : (uint32_t)SEL_OUT);
      plan[PL_DST + d] = nxt;
      cur = nxt;
    }
    plan[PL_NPASS] = npass;
    plan[PL_FINAL] = cur;
    const bool in_out = (cur == SEL_OUT) || (inplace && cur == SEL_IN);
    plan[PL_COPY] = in_out ? 0u : 1u;
    st_agent(done, 0u);
  }
}

// Checks the lane-order property RANK_ATOMIC relies on: for many address patterns (all lanes on
// one word, few words, many words, partial exec masks), lane l must get back the number of lower
// active lanes that hit the same word.  out[0] is left 0 when every check passes.
__global__ __launch_bounds__(256) void k_lane_order_probe(uint32_t* __restrict__ out, uint32_t rounds) {
  __shared__ uint32_t cnt[4][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t bad = 0u;
  for (uint32_t r = 0; r < rounds; ++r) {
    for (int i = lane; i < 256; i += 64) cnt[w][i] = 0u;
    __builtin_amdgcn_wave_barrier();
    // pattern: address from a hash of (round, wave, lane) reduced to 1..256 distinct words
    uint32_t x = (r * 0x9E3779B9u) ^ ((uint32_t)(blockIdx.x * 4 + w) * 0x85EBCA6Bu) ^ ((uint32_t)lane * 0xC2B2AE35u);
    x ^= x >> 15; x *= 0x2C1B3C6Du; x ^= x >> 12;
    const uint32_t span = 1u << (r % 9);                 // 1, 2, 4, ..., 256 distinct words
    const uint32_t a = x & (span - 1u);
    const bool act = ((r % 5) != 4) || ((x >> 20) & 1u);  // every fifth round: random exec mask
    uint32_t got = 0u;
    if (act) got = __hip_atomic_fetch_add(&cnt[w][a], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    // expected rank: active lower lanes with the same word
    uint32_t want = 0u;
    for (int l = 0; l < 64; ++l) {
      const uint32_t al = __shfl(a, l, 64);
      const bool actl = __shfl((int)act, l, 64) != 0;
      want += (l < lane && actl && al == a) ? 1u : 0u;
    }
    if (act && got != want) bad = 1u;
    __builtin_amdgcn_wave_barrier();
  }
  if (bad) atomicOr(out, 1u);
}

// ------------------------------------------------------------------------------------------------
// A3-A6: one digit pass, one workgroup per tile (pass_tile in apsort_pass_core.h).  The tile id is
// claimed from an atomic counter while the LDS counters are cleared, so tiles start in id order
// and the look-back of a tile only waits on tiles that are already running.
// ------------------------------------------------------------------------------------------------
// NT_STORE, NT_LOAD_KV: cache hints of the keys-only scatter and of the pairs' loads (pass_tile).
template <int BITS, int WAVES, int IPT, int RANK, int LB_WIN = 4, bool KV = false, bool NT_STORE = true,
          bool NT_LOAD_KV = false>
__global__ __launch_bounds__(WAVES * 64) void k_pass(
    const uint32_t* in, uint32_t* out, uint32_t* tmp, uint32_t n, int d,
    const uint32_t* __restrict__ plan, const uint32_t* __restrict__ g_base,
    uint32_t* __restrict__ status, uint32_t* __restrict__ tile_ctr, const uint32_t* vin, uint32_t* vout,
    uint32_t* vtmp) {
  if (plan[PL_RUN + d] == 0u) return;
  const uint32_t ssel = plan[PL_SRC + d], dsel = plan[PL_DST + d];
  const uint32_t* src = ssel == SEL_IN ? in : (ssel == SEL_OUT ? out : tmp);
  uint32_t* dst = dsel == SEL_OUT ? out : tmp;
  // values (pairs only) live in the matching buffers and move exactly as their keys
  const uint32_t* vsrc = ssel == SEL_IN ? vin : (ssel == SEL_OUT ? vout : vtmp);
  uint32_t* vdst = dsel == SEL_OUT ? vout : vtmp;
  AP_PASS_SMEM(sm, BITS, WAVES, IPT, RANK, KV);
  __shared__ uint32_t s_tile;
  // the tile claim's round trip overlaps the clearing of the counters; one barrier covers both
  if (threadIdx.x == 0) s_tile = add_agent(tile_ctr + d, 1u);
  pass_clear(sm);
  __syncthreads();
  pass_tile<BITS, WAVES, IPT, RANK, LB_WIN, KV, PASS_DBG_NONE, NT_STORE, NT_LOAD_KV>(
      sm, src, dst, vsrc, vdst, n, s_tile, d * BITS, g_base, status, (int)threadIdx.x);
}

// k_pass (keys only) with a debug mode of pass_tile (PassDebug): seeded timing perturbation, or
// per-tile phase timestamps.  Launched instead of k_pass only while ap_debug_pass is set.
template <int BITS, int WAVES, int IPT, int RANK, int DBG>
__global__ __launch_bounds__(WAVES * 64) void k_pass_dbg(
    const uint32_t* in, uint32_t* out, uint32_t* tmp, uint32_t n, int d, const uint32_t* __restrict__ plan,
    const uint32_t* __restrict__ g_base, uint32_t* __restrict__ status, uint32_t* __restrict__ tile_ctr,
    PassDebugArgs dbg) {
  if (plan[PL_RUN + d] == 0u) return;
  const uint32_t ssel = plan[PL_SRC + d], dsel = plan[PL_DST + d];
  const uint32_t* src = ssel == SEL_IN ? in : (ssel == SEL_OUT ? out : tmp);
  uint32_t* dst = dsel == SEL_OUT ? out : tmp;
  AP_PASS_SMEM(sm, BITS, WAVES, IPT, RANK, false);
  __shared__ uint32_t s_tile;
  if (threadIdx.x == 0) s_tile = add_agent(tile_ctr + d, 1u);
  pass_clear(sm);
  __syncthreads();
  const uint32_t tile = s_tile;
  if constexpr (DBG == PASS_DBG_TRACE) dbg_stamp(dbg, tile, 0);
  if constexpr (DBG == PASS_DBG_PERTURB) dbg_delay(dbg, tile, d * BITS, 0);
  pass_tile<BITS, WAVES, IPT, RANK, 4, false, DBG>(sm, src, dst, nullptr, nullptr, n, tile, d * BITS, g_base, status,
                                                   (int)threadIdx.x, &dbg);
}

// ------------------------------------------------------------------------------------------------
// A7: output contract.  Copies the sorted keys into the output when no pass wrote it, and writes
// splitter p-1 = first key of cell p (all-ones for an empty cell).
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ void copy_u32(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, size_t n,
                                         size_t gtid, size_t gstride) {
  if ((((uintptr_t)src | (uintptr_t)dst) & 15u) == 0u) {
    const uint4* __restrict__ s = reinterpret_cast<const uint4*>(src);
    uint4* __restrict__ o = reinterpret_cast<uint4*>(dst);
    const size_t nv = n >> 2;
    for (size_t i = gtid; i < nv; i += gstride) o[i] = s[i];
    for (size_t i = nv * 4 + gtid; i < n; i += gstride) dst[i] = src[i];
  } else {
    for (size_t i = gtid; i < n; i += gstride) dst[i] = src[i];
  }
}

// vout != nullptr: pairs; their values are copied along with the keys.
__global__ void k_finalize(const uint32_t* in, uint32_t* out, const uint32_t* tmp, uint32_t n,
                           const uint32_t* __restrict__ plan, uint32_t P, uint32_t* __restrict__ splitters,
                           const uint32_t* vin, uint32_t* vout, const uint32_t* vtmp) {
  const uint32_t fsel = plan[PL_FINAL];
  const uint32_t* __restrict__ fin = fsel == SEL_IN ? in : (fsel == SEL_OUT ? out : tmp);
  const size_t gtid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t gstride = (size_t)gridDim.x * blockDim.x;
  if (plan[PL_COPY]) {
    copy_u32(fin, out, n, gtid, gstride);
    if (vout) copy_u32(fsel == SEL_IN ? vin : (fsel == SEL_OUT ? vout : vtmp), vout, n, gtid, gstride);
  }
  if (splitters) {
    const uint64_t q = n / P, r = n % P;
    for (size_t p = gtid + 1; p < P; p += gstride) {
      const uint64_t start = p * q + (p < r ? p : r);
      splitters[p - 1] = start < n ? fin[start] : 0xFFFFFFFFu;
    }
  }
}

}  // namespace aps
