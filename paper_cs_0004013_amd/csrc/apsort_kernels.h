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
//                 communicate, so placement here is exact), and a scatter staged through LDS.
//   k_finalize    Sec. 1.1 output contract: copy when no pass wrote the output, and the P-1
//                 splitters (first key of each cell, footnote to Sec. 3.4.2 for uneven counts).
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

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

// ------------------------------------------------------------------------------------------------
// A1 + A2: bucket counts of all digits in one read, then (last workgroup) constant-digit flags,
// exclusive scans and the pass plan.
//   g_hist   D*R counters, zero on entry, left zero on exit (the last workgroup clears them)
//   done     workgroup-completion counter, zero on entry and on exit
//   zero_ptr/zero_words  scan state of the passes (tile counters + status words), cleared here
//   out_hist optional copy of the final counts (inspection entry point)
// ------------------------------------------------------------------------------------------------
template <int BITS, int THREADS>
__global__ __launch_bounds__(THREADS) void k_hist_plan(
    const uint32_t* __restrict__ keys, uint32_t n, uint32_t* __restrict__ g_hist,
    uint32_t* __restrict__ g_base, uint32_t* __restrict__ plan, uint32_t* __restrict__ done,
    uint4* __restrict__ zero_ptr, uint32_t zero_vec4, int inplace, uint32_t* __restrict__ out_hist) {
  constexpr int R = 1 << BITS;
  constexpr int D = (32 + BITS - 1) / BITS;
  constexpr int HW = D * R;
  __shared__ uint32_t h[HW];
  __shared__ uint32_t s_const[kMaxDigits];
  __shared__ uint32_t s_scan[THREADS / 64];
  __shared__ int s_last;

  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < HW; i += THREADS) h[i] = 0u;
  const uint32_t gtid = blockIdx.x * THREADS + tid, gstride = gridDim.x * THREADS;
  for (uint32_t i = gtid; i < zero_vec4; i += gstride) zero_ptr[i] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();

  auto count = [&](uint32_t k) {
#pragma unroll
    for (int d = 0; d < D; ++d) atomicAdd(&h[d * R + ((k >> (d * BITS)) & (R - 1))], 1u);
  };
  uint32_t head = (uint32_t)(((16u - ((uintptr_t)keys & 15u)) & 15u) >> 2);
  if (head > n) head = n;
  if (gtid < head) count(keys[gtid]);
  const uint4* __restrict__ v = reinterpret_cast<const uint4*>(keys + head);
  const uint32_t nv = (n - head) >> 2;
  uint32_t i = gtid;
  for (; i + 3 * gstride < nv; i += 4 * gstride) {
    const uint4 a = v[i], b = v[i + gstride], c = v[i + 2 * gstride], e = v[i + 3 * gstride];
    count(a.x); count(a.y); count(a.z); count(a.w);
    count(b.x); count(b.y); count(b.z); count(b.w);
    count(c.x); count(c.y); count(c.z); count(c.w);
    count(e.x); count(e.y); count(e.z); count(e.w);
  }
  for (; i < nv; i += gstride) {
    const uint4 a = v[i];
    count(a.x); count(a.y); count(a.z); count(a.w);
  }
  for (uint32_t j = head + nv * 4 + gtid; j < n; j += gstride) count(keys[j]);
  __syncthreads();
  for (uint32_t j = tid; j < HW; j += THREADS) {
    const uint32_t c = h[j];
    if (c) add_agent(&g_hist[j], c);
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = (add_agent(done, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  // ---- last workgroup: every count is in g_hist ----
  if (tid < kMaxDigits) s_const[tid] = 0u;
  __syncthreads();
  for (uint32_t j = tid; j < HW; j += THREADS) {
    const uint32_t c = ld_agent(&g_hist[j]);
    h[j] = c;
    st_agent(&g_hist[j], 0u);
    if (out_hist) out_hist[j] = c;
    if (c == n) s_const[j / R] = 1u;  // one bucket holds every key: the digit is constant
  }
#pragma unroll 1
  for (int d = 0; d < D; ++d) {
    lds_exclusive_scan<R, THREADS>(h + d * R, s_scan);
    for (uint32_t j = tid; j < R; j += THREADS) g_base[d * R + j] = h[d * R + j];
  }
  if (tid == 0) {
    uint32_t npass = 0;
    for (int d = 0; d < D; ++d) npass += s_const[d] ? 0u : 1u;
    // Ping-pong so that the last pass that runs writes the output: with an odd number of passes
    // the first one writes the output, with an even number it writes the scratch buffer.  In
    // place (in == out) the first pass must not write the input, so it always writes scratch.
    const uint32_t first_dst = inplace ? (uint32_t)SEL_TMP : ((npass & 1u) ? (uint32_t)SEL_OUT : (uint32_t)SEL_TMP);
    uint32_t cur = SEL_IN;
    for (int d = 0; d < kMaxDigits; ++d) {
      const uint32_t run = (d < D && !s_const[d]) ? 1u : 0u;
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

// ------------------------------------------------------------------------------------------------
// A3-A6: one digit pass over one tile of T = WAVES*64*IPT keys.
// Keys are taken wave-striped (key j of lane l of wave w sits at w*64*IPT + j*64 + l), which is
// memory order in (w, j, l) order, so ranking sub-step j of every wave in order is stable.
// ------------------------------------------------------------------------------------------------
template <int BITS, int WAVES, int IPT>
__global__ __launch_bounds__(WAVES * 64) void k_pass(
    const uint32_t* in, uint32_t* out, uint32_t* tmp, uint32_t n, int d,
    const uint32_t* __restrict__ plan, const uint32_t* __restrict__ g_base,
    uint32_t* __restrict__ status, uint32_t* __restrict__ tile_ctr) {
  constexpr int R = 1 << BITS;
  constexpr int THREADS = WAVES * 64;
  constexpr int T = THREADS * IPT;
  constexpr int BPT = (R + THREADS - 1) / THREADS;
  if (plan[PL_RUN + d] == 0u) return;
  const uint32_t ssel = plan[PL_SRC + d], dsel = plan[PL_DST + d];
  const uint32_t* __restrict__ src = ssel == SEL_IN ? in : (ssel == SEL_OUT ? out : tmp);
  uint32_t* __restrict__ dst = dsel == SEL_OUT ? out : tmp;
  const int shift = d * BITS;

  __shared__ uint32_t s_cnt[WAVES * R];  // per-wave bucket counters, then per-wave start offsets
  __shared__ uint32_t s_delta[R];        // bucket totals -> tile-local bucket starts -> global delta
  __shared__ uint32_t s_stage[T];        // keys in tile-sorted order
  __shared__ uint32_t s_scan[THREADS / 64];
  __shared__ uint32_t s_tile;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_tile = add_agent(tile_ctr + d, 1u);
  for (int j = tid; j < WAVES * R; j += THREADS) s_cnt[j] = 0u;
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint32_t tbase = tile * (uint32_t)T;

  // ---- load: keys past n become all-ones sentinels (largest digit, last in order) ----
  uint32_t k[IPT];
  const uint32_t wbase = tbase + (uint32_t)(wid * 64 * IPT + lane);
  if (tbase + (uint32_t)T <= n) {
#pragma unroll
    for (int j = 0; j < IPT; ++j) k[j] = src[wbase + j * 64];
  } else {
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const uint32_t idx = wbase + j * 64;
      k[j] = idx < n ? src[idx] : 0xFFFFFFFFu;
    }
  }

  // ---- A4: stable rank within the wave's keys ----
  uint32_t r[IPT];
  uint32_t* cnt = s_cnt + wid * R;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint32_t v = (k[j] >> shift) & (R - 1);
    const uint64_t m = match_any<BITS>(v);
    const uint32_t peers = lanes_below(m);
    const uint32_t c = cnt[v];
    r[j] = c + peers;
    if (peers == 0u) cnt[v] = c + (uint32_t)__popcll(m);
  }
  __syncthreads();

  // ---- tile bucket totals; publish them for the look-back of later tiles ----
  uint32_t tot[BPT];
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int b = tid + i * THREADS;
    tot[i] = 0u;
    if (b < R) {
      uint32_t s = 0u;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = s_cnt[w * R + b];
        s_cnt[w * R + b] = s;
        s += c;
      }
      tot[i] = s;
      s_delta[b] = s;
      if (tile == 0u) st_agent(status + b, kFlagPrefix | (g_base[b] + s));
      else st_agent(status + (size_t)tile * R + b, kFlagAgg | s);
    }
  }
  lds_exclusive_scan<R, THREADS>(s_delta, s_scan);  // s_delta = tile-local bucket starts

  // ---- A3: decoupled look-back for each bucket's global start ----
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int b = tid + i * THREADS;
    if (b < R) {
      uint32_t excl;
      if (tile == 0u) {
        excl = g_base[b];
      } else {
        excl = 0u;
        uint32_t p = tile - 1;
        while (true) {
          const uint32_t s = ld_agent(status + (size_t)p * R + b);
          const uint32_t f = s & kFlagMask;
          if (f == 0u) {
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          excl += s & kValueMask;
          if (f == kFlagPrefix) break;
          --p;
        }
        st_agent(status + (size_t)tile * R + b, kFlagPrefix | (excl + tot[i]));
      }
      const uint32_t lb = s_delta[b];
#pragma unroll
      for (int w = 0; w < WAVES; ++w) s_cnt[w * R + b] += lb;
      s_delta[b] = excl - lb;
    }
  }
  __syncthreads();

  // ---- A5: reorder through LDS, then coalesced scatter ----
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint32_t v = (k[j] >> shift) & (R - 1);
    s_stage[cnt[v] + r[j]] = k[j];
  }
  __syncthreads();
  const uint32_t nvalid = (n - tbase) < (uint32_t)T ? (n - tbase) : (uint32_t)T;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint32_t i = (uint32_t)(j * THREADS + tid);
    if (i < nvalid) {
      const uint32_t key = s_stage[i];
      const uint32_t v = (key >> shift) & (R - 1);
      dst[s_delta[v] + i] = key;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// A7: output contract.  Copies the sorted keys into the output when no pass wrote it, and writes
// splitter p-1 = first key of cell p (all-ones for an empty cell).
// ------------------------------------------------------------------------------------------------
__global__ void k_finalize(const uint32_t* in, uint32_t* out, const uint32_t* tmp, uint32_t n,
                           const uint32_t* __restrict__ plan, uint32_t P, uint32_t* __restrict__ splitters) {
  const uint32_t fsel = plan[PL_FINAL];
  const uint32_t* __restrict__ fin = fsel == SEL_IN ? in : (fsel == SEL_OUT ? out : tmp);
  const size_t gtid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t gstride = (size_t)gridDim.x * blockDim.x;
  if (plan[PL_COPY]) {
    if ((((uintptr_t)fin | (uintptr_t)out) & 15u) == 0u) {
      const uint4* __restrict__ s = reinterpret_cast<const uint4*>(fin);
      uint4* __restrict__ o = reinterpret_cast<uint4*>(out);
      const size_t nv = n >> 2;
      for (size_t i = gtid; i < nv; i += gstride) o[i] = s[i];
      for (size_t i = nv * 4 + gtid; i < n; i += gstride) out[i] = fin[i];
    } else {
      for (size_t i = gtid; i < n; i += gstride) out[i] = fin[i];
    }
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
