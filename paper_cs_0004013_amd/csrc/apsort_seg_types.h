// Data structures shared by the segmented-sort kernels and their host callers.
#pragma once

#include <stdint.h>

namespace aps {

constexpr int kSegBuckets = 32;  // work-list classes: ceil(log2(length))
constexpr int kSegGroups = 6;    // length groups, each sorted by its own kernel configuration

// Control block of the segmented sort (device memory, zero between calls).
struct SegCtl {
  uint32_t count[kSegBuckets];   // segments per length class
  uint32_t start[kSegBuckets];   // first slot of each class in the work order (longest first)
  uint32_t cursor[kSegBuckets];  // fill cursors
  uint32_t nwork;                // segments to sort (length >= 2 and valid)
  uint32_t done;                 // completion counter of k_seg_classify's last-workgroup pattern
  uint32_t bad;                  // 1 when some offsets were invalid
  uint32_t pad0;
  uint32_t head[kSegGroups];     // next work item of each length group's kernel
  uint32_t done2[kSegGroups];    // exit counters of each group's kernel
  // long segments (sorted by device-wide passes over one flat tile space)
  unsigned long long long_cursor;  // (long segments << 32) | flat tiles, advanced by k_seg_fill
  uint32_t long_ctr[4];            // tile claim counters of the four digit passes
};

// A long segment: keys[0..n) sorted in place by device-wide digit passes, through tmp[0..n); its
// tiles are flat tiles [first_tile, first_tile + ntiles) of the batch.  The plan is written by
// k_seg_long_plan from the segment's bucket counts.
struct LongSeg {
  uint32_t* keys;
  uint32_t* tmp;
  uint32_t n;
  uint32_t first_tile;
  uint32_t ntiles;
  uint32_t npass;       // digit passes that run
  uint32_t run[4];      // pass d runs (its digit is not constant over the segment)
  uint32_t rd_tmp[4];   // pass d reads tmp and writes keys (else reads keys, writes tmp)
  uint32_t final_tmp;   // the sorted keys end in tmp and are copied back
  uint32_t pad[3];
};

// One unit of work of the persistent sort: sort src[0..n) into dst[0..n) (src == dst allowed),
// using tmp[0..n) as scratch when more than one tile is needed; when spl is not NULL also write
// the P-1 splitters of the n sorted keys spread over P cells.
struct SegDesc {
  const uint32_t* src;
  uint32_t* dst;
  uint32_t* tmp;
  uint32_t* spl;
  uint32_t n;
  uint32_t P;
  uint32_t pad[2];
};

}  // namespace aps
