/*
 * Plain C consumer of libapsort.so: device memory from the HIP runtime's C API, every sort call
 * through include/apsort.h, results checked on the host.  Exit status 0 and the line "consumer ok"
 * on success.  Test program only.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "apsort.h"

#define CHECK_HIP(x)                                                       \
  do {                                                                     \
    hipError_t e_ = (x);                                                   \
    if (e_ != hipSuccess) {                                                \
      fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));      \
      return 1;                                                            \
    }                                                                      \
  } while (0)
#define CHECK_AP(x)                                                        \
  do {                                                                     \
    ap_status s_ = (x);                                                    \
    if (s_ != AP_OK) {                                                     \
      fprintf(stderr, "%s failed (%d): %s\n", #x, (int)s_, ap_last_error()); \
      return 1;                                                            \
    }                                                                      \
  } while (0)

static uint64_t lcg_state = 88172645463325252ull;
static uint32_t rnd31(void) {
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(lcg_state >> 33);
}
static int cmp_u32(const void* a, const void* b) {
  const uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : (x > y);
}

int main(void) {
  const size_t n = 3000017;
  const int P = 64;
  uint32_t* h = (uint32_t*)malloc(n * 4);
  uint32_t* want = (uint32_t*)malloc(n * 4);
  uint32_t* got = (uint32_t*)malloc(n * 4);
  uint32_t spl[63];
  for (size_t i = 0; i < n; ++i) h[i] = rnd31();
  memcpy(want, h, n * 4);
  qsort(want, n, 4, cmp_u32);

  uint32_t *d_in = NULL, *d_out = NULL, *d_spl = NULL, *d_off = NULL, *d_st = NULL;
  CHECK_HIP(hipMalloc((void**)&d_in, n * 4));
  CHECK_HIP(hipMalloc((void**)&d_out, n * 4));
  CHECK_HIP(hipMalloc((void**)&d_spl, 63 * 4));
  CHECK_HIP(hipMemcpy(d_in, h, n * 4, hipMemcpyHostToDevice));

  /* one array, 64 cells */
  CHECK_AP(ap_sort_u32(d_in, d_out, n, P, d_spl, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(got, d_out, n * 4, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(spl, d_spl, 63 * 4, hipMemcpyDeviceToHost));
  if (memcmp(got, want, n * 4) != 0) { fprintf(stderr, "sorted keys differ\n"); return 1; }
  for (int p = 1; p < P; ++p) {
    const size_t q = n / P, r = n % P, start = p * q + ((size_t)p < r ? (size_t)p : r);
    if (spl[p - 1] != want[start]) { fprintf(stderr, "splitter %d wrong\n", p - 1); return 1; }
  }

  /* caller-owned workspace, in place */
  size_t ws_bytes = ap_sort_workspace_bytes(n);
  void* d_ws = NULL;
  CHECK_HIP(hipMalloc(&d_ws, ws_bytes));
  CHECK_AP(ap_workspace_init(d_ws, ws_bytes, NULL));
  CHECK_HIP(hipMemcpy(d_out, h, n * 4, hipMemcpyHostToDevice));
  CHECK_AP(ap_sort_u32_ws(d_out, d_out, n, P, NULL, d_ws, ws_bytes, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(got, d_out, n * 4, hipMemcpyDeviceToHost));
  if (memcmp(got, want, n * 4) != 0) { fprintf(stderr, "in-place workspace sort differs\n"); return 1; }

  /* pairs: values = positions, i.e. an argsort; equal keys keep their input order */
  {
    uint32_t *d_vin = NULL, *d_vout = NULL;
    uint32_t* hv = (uint32_t*)malloc(n * 4);
    for (size_t i = 0; i < n; ++i) {
      h[i] &= 0xFFFFu; /* many equal keys: the order among them is observable */
      hv[i] = (uint32_t)i;
    }
    CHECK_HIP(hipMalloc((void**)&d_vin, n * 4));
    CHECK_HIP(hipMalloc((void**)&d_vout, n * 4));
    CHECK_HIP(hipMemcpy(d_in, h, n * 4, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_vin, hv, n * 4, hipMemcpyHostToDevice));
    CHECK_AP(ap_sort_pairs_u32(d_in, d_vin, d_out, d_vout, n, 1, NULL, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    CHECK_HIP(hipMemcpy(got, d_out, n * 4, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(hv, d_vout, n * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < n; ++i) {
      if (got[i] != h[hv[i]]) { fprintf(stderr, "pairs: value %zu does not belong to its key\n", i); return 1; }
      if (i && (got[i - 1] > got[i] || (got[i - 1] == got[i] && hv[i - 1] >= hv[i]))) {
        fprintf(stderr, "pairs: order or stability broken at %zu\n", i);
        return 1;
      }
    }
    for (size_t i = 0; i < n; ++i) h[i] = rnd31(); /* restore a full-range key set */
    hipFree(d_vin);
    hipFree(d_vout);
    free(hv);
  }

  /* segmented: 7 segments in place */
  uint32_t off[8] = {0, 5, 5, 70000, 70001, 400000, 1234567, (uint32_t)n};
  CHECK_HIP(hipMalloc((void**)&d_off, sizeof off));
  CHECK_HIP(hipMalloc((void**)&d_st, 4));
  CHECK_HIP(hipMemset(d_st, 0, 4));
  CHECK_HIP(hipMemcpy(d_off, off, sizeof off, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_out, h, n * 4, hipMemcpyHostToDevice));
  CHECK_AP(ap_sort_u32_segmented(d_out, n, d_off, 7, d_st, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(got, d_out, n * 4, hipMemcpyDeviceToHost));
  uint32_t st = 1;
  CHECK_HIP(hipMemcpy(&st, d_st, 4, hipMemcpyDeviceToHost));
  if (st != 0) { fprintf(stderr, "segmented status %u\n", st); return 1; }
  memcpy(want, h, n * 4);
  for (int s = 0; s < 7; ++s) qsort(want + off[s], off[s + 1] - off[s], 4, cmp_u32);
  if (memcmp(got, want, n * 4) != 0) { fprintf(stderr, "segmented keys differ\n"); return 1; }

  /* server: three requests, waited for in reverse order */
  ap_server_cfg cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.hbm_budget_bytes = (size_t)1 << 30;
  cfg.num_streams = 2;
  ap_server* srv = NULL;
  CHECK_AP(ap_server_create(&cfg, &srv));
  CHECK_HIP(hipMemcpy(d_in, h, n * 4, hipMemcpyHostToDevice));
  const size_t lens[3] = {1000, 200000, 2000000};
  size_t at = 0;
  uint64_t tk[3];
  for (int i = 0; i < 3; ++i) {
    CHECK_AP(ap_server_submit(srv, d_in + at, d_out + at, lens[i], 1, NULL, &tk[i]));
    at += lens[i];
  }
  for (int i = 2; i >= 0; --i) CHECK_AP(ap_server_wait(srv, tk[i], -1));
  CHECK_AP(ap_server_destroy(srv));
  CHECK_HIP(hipMemcpy(got, d_out, at * 4, hipMemcpyDeviceToHost));
  memcpy(want, h, at * 4);
  at = 0;
  for (int i = 0; i < 3; ++i) {
    qsort(want + at, lens[i], 4, cmp_u32);
    at += lens[i];
  }
  if (memcmp(got, want, at * 4) != 0) { fprintf(stderr, "served keys differ\n"); return 1; }

  /* merge of two sorted runs: into another buffer, and in place as adjacent runs of one array */
  {
    const size_t na = n / 3, nb = n - n / 3;
    memcpy(want, h, n * 4);
    qsort(want, na, 4, cmp_u32);
    qsort(want + na, nb, 4, cmp_u32);
    CHECK_HIP(hipMemcpy(d_out, want, n * 4, hipMemcpyHostToDevice));
    CHECK_AP(ap_merge_u32(d_out, na, d_out + na, nb, d_in, NULL));
    CHECK_AP(ap_merge_adjacent_u32(d_out, na, nb, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    qsort(want, n, 4, cmp_u32);
    CHECK_HIP(hipMemcpy(got, d_in, n * 4, hipMemcpyDeviceToHost));
    if (memcmp(got, want, n * 4) != 0) { fprintf(stderr, "merged runs differ\n"); return 1; }
    CHECK_HIP(hipMemcpy(got, d_out, n * 4, hipMemcpyDeviceToHost));
    if (memcmp(got, want, n * 4) != 0) { fprintf(stderr, "adjacent-run merge differs\n"); return 1; }
  }

  hipFree(d_in); hipFree(d_out); hipFree(d_spl); hipFree(d_off); hipFree(d_st); hipFree(d_ws);
  free(h); free(want); free(got);
  printf("consumer ok (%s)\n", ap_version());
  return 0;
}
