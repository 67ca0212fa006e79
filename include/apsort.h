/*
 * apsort -- radix sort of 32-bit integer keys on MI355X (gfx950).
 *
 * C ABI of libapsort.so.  The method is the radix sort of Weaver & Lynes,
 * "Sorting Integers on the AP1000": keys are bucketed by digit (Sec. 3.2:
 * bucket counts, cumulative totals, partial sort), digit by digit from the
 * least significant one, each pass stable (Sec. 3.3.1), and the sorted keys
 * are then spread evenly over P cells, cell 0 holding the smallest keys
 * (Sec. 1.1), the cells with lower ids taking the extra key when n is not a
 * multiple of P (footnote to Sec. 3.4.2).  On one GPU the cells are P
 * contiguous slices of the output array; the global radix sort over all keys
 * that Sec. 5 analyses is what runs.
 *
 * Conventions for every entry point
 *   - Pointers named d_* are device pointers of the current HIP device.  Keys
 *     are uint32_t and must be 4-byte aligned; no other alignment is assumed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Work is enqueued on it and the call returns right after the
 *     enqueue; results are ready when the stream reaches that point.
 *   - The caller owns every d_* buffer and keeps it alive until the stream
 *     work completes.  Input buffers are never written.
 *   - Argument errors are detected before anything is enqueued and return
 *     AP_ERR_INVALID (nothing is written).  A failed HIP call returns
 *     AP_ERR_HIP, an allocation failure AP_ERR_NOMEM.  ap_last_error() gives a
 *     thread-local message for the last failure.
 *   - Key counts are limited to n < 2^30 per call: the single-pass scan packs a
 *     30-bit running count with a 2-bit state in one 32-bit word.
 */
#ifndef APSORT_H
#define APSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AP_OK = 0,
    AP_ERR_INVALID = 1,    /* bad argument; nothing enqueued */
    AP_ERR_NOMEM = 2,      /* device or host allocation failed */
    AP_ERR_HIP = 3,        /* a HIP runtime call or launch failed */
    AP_ERR_BUDGET = 4,     /* server: request larger than the memory budget */
    AP_ERR_QUEUE_FULL = 5, /* server: submission queue full */
    AP_ERR_TIMEOUT = 6,    /* server: wait timed out / ticket still pending */
    AP_ERR_DEVICE = 7,     /* server: the request's device work failed */
    AP_ERR_CANCELLED = 8   /* server: the server was destroyed before the request ran */
} ap_status;

#define AP_MAX_KEYS ((size_t)1 << 30) /* exclusive upper bound on n per call */

/*
 * ap_sort_u32 -- sort n keys and place them in P equal cells.
 *
 * Computes d_out[0..n) = the keys of d_in[0..n) in nondecreasing unsigned
 * order (the full LSD radix sort: Sec. 3.2 bucketing per digit, Sec. 3.3.1
 * digit order and stability).  Cell p (p = 0..P-1) is the slice
 * [start(p), start(p+1)) with q = n / P, r = n % P, start(p) = p*q + min(p, r)
 * (Sec. 1.1 and the footnote to Sec. 3.4.2).  When d_splitters is not NULL it
 * receives P-1 values: d_splitters[p-1] = d_out[start(p)], the lowest key of
 * cell p, or 0xFFFFFFFF when cell p is empty (n < P; all-ones padding in the
 * spirit of Sec. 2.1.1).
 *
 *   d_in        n keys, read only.  d_in == d_out (in place) is allowed; any
 *               other overlap of the two ranges is AP_ERR_INVALID.
 *   d_out       n keys, written.
 *   n           0 <= n < AP_MAX_KEYS.  n == 0 writes only the splitters.
 *   P           number of cells, P >= 1.
 *   d_splitters P-1 uint32_t, or NULL.
 *
 * Digit columns whose value is the same for every key are not sorted on (the
 * pass is an identity); this is decided on the device, with no host sync.
 * Arrays of at most 16384 keys are sorted in one launch by one workgroup in
 * registers and LDS, with no scratch memory.  Longer ones take the
 * device-wide passes.  Their scratch memory (about 4n bytes plus the scan state)
 * comes from a per-device, per-stream cache that grows on demand; growing
 * synchronises `stream` first.  Use ap_sort_u32_ws to bring your own
 * workspace instead (it always takes the device-wide passes).
 */
ap_status ap_sort_u32(const uint32_t *d_in, uint32_t *d_out, size_t n, int P,
                      uint32_t *d_splitters, void *stream);

/*
 * ap_sort_workspace_bytes -- size of the workspace ap_sort_u32_ws needs for
 * n keys.  Returns 0 when n >= AP_MAX_KEYS.
 */
size_t ap_sort_workspace_bytes(size_t n);

/*
 * ap_workspace_init -- prepare a caller-owned workspace of ws_bytes bytes
 * (zero its control words) on `stream`.  Required once before the first
 * ap_sort_u32_ws call on that memory; every successful sort leaves the
 * workspace ready for the next one.
 */
ap_status ap_workspace_init(void *d_ws, size_t ws_bytes, void *stream);

/*
 * ap_sort_u32_ws -- ap_sort_u32 with a caller-owned workspace
 * (d_ws, ws_bytes >= ap_sort_workspace_bytes(n), 256-byte aligned, prepared
 * once by ap_workspace_init).  Performs no allocation and no host
 * synchronisation.  Two calls that overlap in time must not share d_ws.
 */
ap_status ap_sort_u32_ws(const uint32_t *d_in, uint32_t *d_out, size_t n, int P,
                         uint32_t *d_splitters, void *d_ws, size_t ws_bytes,
                         void *stream);

/*
 * ap_sort_u32_msd -- ap_sort_u32 organised as bucketing on the high-order
 * bits followed by a local sort of every bucket (Sec. 3.2 bucketing on the
 * top bits with 4096, then 8192 buckets, Sec. 4.7; Sec. 3.3 local radix sort
 * per cell) instead of one least-significant-digit pass per digit.  Same
 * arguments, results and errors as ap_sort_u32.
 *
 * The keys are ordered by their top 16 bits (2^16 buckets) with the two
 * high-order device-wide digit passes, the bucket boundaries are found by
 * binary search, and the buckets are sorted in place by the batched
 * segmented sort (one workgroup per bucket in LDS; buckets of the
 * long-segment size and more by device-wide passes), then the splitters are
 * written.  Scratch: the ap_sort_u32 cache of the stream plus 256 KiB, and
 * the segmented sort's cache of the stream.
 */
ap_status ap_sort_u32_msd(const uint32_t *d_in, uint32_t *d_out, size_t n, int P,
                          uint32_t *d_splitters, void *stream);

/*
 * ap_sort_u32_noalloc -- ap_sort_u32 for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as ap_sort_u32, with
 * n <= AP_NOALLOC_MAX_KEYS (larger n: AP_ERR_INVALID, nothing enqueued).
 *
 * Its scratch is a fixed 26 MiB array in the library's device memory, which
 * every GPU the library runs on holds until the process ends.  The call makes
 * no allocation, no host synchronisation and no memset (the array's control
 * words are zeroed by a kernel on `stream`), so it can be captured.  All calls
 * on one device share that array and the previous call's contents are
 * overwritten: calls that overlap in time on one device (other streams, other
 * threads) race and must be serialised by the caller.  The rank primitive is
 * the atomic one only if another entry point has already run the device's
 * lane-order check (see ap_rank_check_state); otherwise the order-agnostic
 * rank runs, with identical results.
 */
#define AP_NOALLOC_MAX_KEYS ((size_t)1 << 22)
ap_status ap_sort_u32_noalloc(const uint32_t *d_in, uint32_t *d_out, size_t n,
                              int P, uint32_t *d_splitters, void *stream);

/*
 * ap_sort_pairs_u32 -- sort (key, value) pairs by key.
 *
 * The same LSD radix sort on the keys (Sec. 3.2 bucketing per digit, Sec.
 * 3.3.1 digit order), every 32-bit value moving with its key.  Every pass
 * keeps the order of elements with equal digits (Sec. 3.3.1), so pairs with
 * equal keys leave in their input order: with values 0..n-1 the output values
 * are the stable sorting permutation (an argsort).  The keys, cells and
 * splitters are exactly those of ap_sort_u32 on d_keys_in.
 *   d_keys_in, d_vals_in    n keys and n values (never written unless in place)
 *   d_keys_out, d_vals_out  n sorted keys and their values
 * In place is allowed when d_keys_in == d_keys_out and d_vals_in ==
 * d_vals_out (both, or neither: AP_ERR_INVALID otherwise); a key array must
 * not overlap a value array.  Tiles are at most 16K keys (keys and values are
 * both staged in LDS).  Scratch (about 8n bytes plus the scan state) comes
 * from the same per-stream cache as ap_sort_u32.
 */
ap_status ap_sort_pairs_u32(const uint32_t *d_keys_in, const uint32_t *d_vals_in,
                            uint32_t *d_keys_out, uint32_t *d_vals_out, size_t n,
                            int P, uint32_t *d_splitters, void *stream);

/*
 * ap_sort_pairs_workspace_bytes / ap_sort_pairs_u32_ws -- the pairs sort with
 * a caller-owned workspace (prepared once by ap_workspace_init, 256-byte
 * aligned, at least ap_sort_pairs_workspace_bytes(n) bytes); no allocation,
 * no host synchronisation.  Returns 0 bytes when n >= AP_MAX_KEYS.
 */
size_t ap_sort_pairs_workspace_bytes(size_t n);
ap_status ap_sort_pairs_u32_ws(const uint32_t *d_keys_in, const uint32_t *d_vals_in,
                               uint32_t *d_keys_out, uint32_t *d_vals_out, size_t n,
                               int P, uint32_t *d_splitters, void *d_ws,
                               size_t ws_bytes, void *stream);

/*
 * ap_merge_u32 -- merge two sorted runs: the merge step of the merge-exchange
 * (Sec. 3.4: two sorted lists merged in the classic manner; the cell with the
 * lower id keeps the lower values).
 *   d_a, na   keys in nondecreasing order (unsigned)
 *   d_b, nb   keys in nondecreasing order
 *   d_out     na + nb keys: the merged, nondecreasing sequence; equal keys
 *             from d_a come before those from d_b.  d_out[0..na) and
 *             d_out[na..na+nb) are the two cells' parts after a merge-exchange.
 * na + nb < 2^30; d_out must not overlap an input (AP_ERR_INVALID).  Inputs that
 * are not sorted give an unspecified permutation of the keys (nothing outside
 * d_out is written).  Scratch (one word per 4096 outputs) comes from a
 * per-stream cache.
 */
ap_status ap_merge_u32(const uint32_t *d_a, size_t na, const uint32_t *d_b,
                       size_t nb, uint32_t *d_out, void *stream);

/*
 * ap_merge_adjacent_u32 -- merge the sorted runs d_keys[0..na) and
 * d_keys[na..na+nb) of one array in place (Sec. 4.6: the two sorted lists of
 * one cell's array merged into one).  The runs are copied to per-stream
 * scratch (4(na+nb) bytes) and merged back.
 */
ap_status ap_merge_adjacent_u32(uint32_t *d_keys, size_t na, size_t nb, void *stream);

/*
 * ap_digit_plan_u32 -- the first step of the sort on its own, for inspection:
 * the bucket counts of every digit (Sec. 3.2, first loop of bucket()) and the
 * pass plan derived from them.
 *
 *   digit_bits  digit width b, 4 <= b <= 11; D = ceil(32 / b) digits.
 *   d_hist      D * 2^b uint32_t; d_hist[d * 2^b + v] = number of keys whose
 *               digit d ((key >> (b*d)) & (2^b - 1)) equals v.
 *   d_plan      D + 1 uint32_t, or NULL: d_plan[d] = 1 when pass d runs (its
 *               digit is not constant over the keys), 0 when it is skipped;
 *               d_plan[D] = number of passes that run.
 */
ap_status ap_digit_plan_u32(const uint32_t *d_in, size_t n, int digit_bits,
                            uint32_t *d_hist, uint32_t *d_plan, void *stream);

/*
 * ap_sort_u32_segmented -- sort many independent arrays (segments) of one
 * buffer in place, in one launch sequence.
 *
 * Segment s is d_keys[d_offsets[s] .. d_offsets[s+1]), s = 0..nseg-1; each is
 * sorted independently into nondecreasing order, as each AP1000 cell sorts
 * its own keys in the local-sort phase (Sec. 3.3, LSD radix sort of
 * Sec. 3.3.1).  Keys outside every segment are not touched.
 *
 *   d_keys     n_total keys (device), sorted in place segment by segment.
 *   n_total    number of keys in d_keys, < AP_MAX_KEYS; every offset must be
 *              <= n_total.
 *   d_offsets  nseg + 1 uint32_t offsets (device), nondecreasing.
 *   nseg       number of segments, >= 0.
 *   d_status   optional device uint32_t: set to 0 when the offsets are valid,
 *              to AP_ERR_INVALID when some offset decreases or exceeds n_total;
 *              then no segment is sorted (invalid offsets make segments
 *              overlap).  The offsets live on the device, so this check
 *              completes with the stream work rather than at the call.
 *
 * Segments shorter than the long-segment threshold (ap_segmented_set_long_min,
 * default 2^20 keys) are sorted by one workgroup each: segments that fit one
 * tile in registers and LDS (one read and one write of each key); longer ones
 * by the same workgroup with a histogram sweep and one sweep per non-constant
 * digit; they are scheduled longest first by persistent kernels, one per
 * length group.  Segments at or above the threshold are sorted like one
 * array, by device-wide digit passes (bucket counts per segment, then one pass
 * per non-constant digit with a single-pass scan over the tiles of all long
 * segments), beside the workgroup-per-segment kernels.  No host
 * synchronisation; on a non-default stream the launch sequence is captured
 * into a hipGraph and replayed while the arguments repeat.  Scratch memory
 * (ap_segmented_workspace_bytes: 4 * n_total bytes + 32 bytes per segment,
 * plus, when long segments are possible, about 1 KiB per 256 keys) is cached
 * per device and stream.
 */
ap_status ap_sort_u32_segmented(uint32_t *d_keys, size_t n_total,
                                const uint32_t *d_offsets, int nseg,
                                uint32_t *d_status, void *stream);

/*
 * ap_segmented_set_long_min / ap_segmented_get_long_min -- segments of at
 * least long_min keys are sorted by the device-wide passes (0 = never; 1 is
 * AP_ERR_INVALID).  Process-wide; results do not depend on it.
 */
ap_status ap_segmented_set_long_min(size_t long_min);
size_t ap_segmented_get_long_min(void);

/* ap_segmented_workspace_bytes -- scratch size of a segmented call. */
size_t ap_segmented_workspace_bytes(size_t n_total, int nseg);

/*
 * Segmented-sort tuning.  Segments (and batched server requests) fall in
 * length groups: group g covers the lengths whose length class, ceil(log2(length))
 * (lengths 0..2 count as class 1), lies in [cls_lo, cls_hi] and runs kernel
 * configuration cfg (digit width, waves per
 * workgroup, keys per lane; ap_segmented_num_configs() configurations are
 * compiled in, see ap_segmented_config_info).  A group with cls_lo > cls_hi
 * is unused; the used groups must cover every class 1..31 exactly once.
 * ap_load_tuning rejects a table that does not (AP_ERR_INVALID, nothing
 * installed); a table built group by group with ap_segmented_set_group is
 * checked when a segmented sort or a server batch is launched, which then
 * fails with AP_ERR_INVALID (nothing enqueued; for the server, every request
 * of the batch completes with AP_ERR_DEVICE).  Settings are process-wide.
 *   ap_segmented_set_config(cfg)  every group uses cfg
 *   ap_segmented_set_group / ap_segmented_get_group  one group
 *   ap_load_tuning(path)  replace the table from a text file with lines
 *                         "group cls_lo cls_hi cfg" ('#' starts a comment),
 *                         as written by the package's autotuner
 */
int ap_segmented_num_configs(void);
int ap_segmented_num_groups(void);  /* number of length groups g */
ap_status ap_segmented_config_info(int cfg, int *digit_bits, int *waves,
                                   int *keys_per_lane);
ap_status ap_segmented_set_config(int cfg);
ap_status ap_segmented_set_group(int g, int cls_lo, int cls_hi, int cfg);
ap_status ap_segmented_get_group(int g, int *cls_lo, int *cls_hi, int *cfg);
ap_status ap_load_tuning(const char *path);

/*
 * Request server: sort requests from any number of host threads, batched as
 * they arrive (continuous batching) and run on several streams at once.
 *
 * A request has the contract of ap_sort_u32 (d_in, d_out, n, P, splitters).
 * Submission is non-blocking and returns a ticket; the request is queued,
 * admitted when its scratch fits the memory budget of a free slot, and run:
 * requests shorter than alone_min_keys are batched into one launch of the
 * persistent segmented kernel (each request sorted by one workgroup, straight
 * from its input to its output buffer), longer ones run alone through the
 * device-wide sort.  Requests that arrive while slots are busy join the next
 * batch formed on a slot that frees up.  The caller keeps every buffer alive
 * until its ticket completes.
 *
 *   hbm_budget_bytes  scratch memory of the server: one arena allocated at
 *                     creation and shared by all slots; default 64 GiB.  It is
 *                     kept as a ledger: a batch or a long request reserves the
 *                     byte range it needs (first fit) when it is launched and
 *                     returns it when it completes, so a long request may use
 *                     nearly all of it.  A long request at the queue head that
 *                     does not fit yet waits, and meanwhile only requests that
 *                     need no scratch (at most 2048 keys) are launched.
 *   num_streams       slots = concurrent batches; default 4.
 *   max_batch         requests per batch; default 256.
 *   max_queue         queued requests before AP_ERR_QUEUE_FULL; default 65536.
 *   alone_min_keys    requests with n >= this run alone; default 2^16 (one
 *                     workgroup per request is slower than the device-wide
 *                     sort above that size).
 * Zero fields take the default.
 *
 * ap_server_submit: AP_ERR_INVALID for bad arguments, AP_ERR_BUDGET when the
 *   request's scratch exceeds the whole budget (it could never run),
 *   AP_ERR_QUEUE_FULL when the queue is full.  Nothing is queued then.
 * ap_server_wait: the ticket's final status (AP_OK, AP_ERR_DEVICE when its
 *   device work failed, AP_ERR_CANCELLED when the server was destroyed before
 *   it ran), or AP_ERR_TIMEOUT after timeout_us microseconds (< 0: no limit).
 *   A ticket whose final status has been returned is forgotten.
 * ap_server_poll: like ap_server_wait with a zero timeout.
 * ap_server_get_stats: counters, submit-to-completion latency and
 *   submit-to-launch queueing percentiles of the completed requests (since
 *   creation or the last reset), and the scratch arena's size and peak use
 *   (since creation).
 * ap_server_destroy: cancels queued requests, waits for running ones, frees
 *   everything.  No other call on the server may run concurrently with it.
 * ap_server_submit_flags: ap_server_submit with flags; AP_SUBMIT_INJECT_FAULT
 *   (testing) makes that one request fail with AP_ERR_DEVICE without running.
 * ap_server_submit_at: ap_server_submit_flags for a request that arrived at
 *   arrival_ns (nanoseconds on CLOCK_MONOTONIC, as clock_gettime gives it; 0
 *   or a time in the future = now).  The latency statistics of the request
 *   then run from its arrival rather than from the call, so time a client
 *   spent before it could submit is counted.
 */
typedef struct {
    size_t hbm_budget_bytes;
    int num_streams;
    int max_batch;
    int max_queue;
    size_t alone_min_keys;
} ap_server_cfg;

typedef struct {
    uint64_t submitted, completed, failed, cancelled, batches, alone, keys;
    uint64_t latency_samples;
    double p50_us, p99_us, mean_us, max_us;
    double queue_p50_us, queue_p99_us;  /* submit (or arrival) to launch */
    uint64_t scratch_budget_bytes;      /* size of the shared scratch arena */
    uint64_t scratch_peak_bytes;        /* most scratch reserved at once */
} ap_server_stats;

typedef struct ap_server ap_server;

#define AP_SUBMIT_INJECT_FAULT 1u

ap_status ap_server_create(const ap_server_cfg *cfg, ap_server **out);
ap_status ap_server_submit(ap_server *s, const uint32_t *d_in, uint32_t *d_out,
                           size_t n, int P, uint32_t *d_splitters,
                           uint64_t *ticket);
ap_status ap_server_submit_flags(ap_server *s, const uint32_t *d_in,
                                 uint32_t *d_out, size_t n, int P,
                                 uint32_t *d_splitters, unsigned flags,
                                 uint64_t *ticket);
ap_status ap_server_submit_at(ap_server *s, const uint32_t *d_in,
                              uint32_t *d_out, size_t n, int P,
                              uint32_t *d_splitters, unsigned flags,
                              uint64_t arrival_ns, uint64_t *ticket);
ap_status ap_server_wait(ap_server *s, uint64_t ticket, int64_t timeout_us);
ap_status ap_server_poll(ap_server *s, uint64_t ticket);
ap_status ap_server_get_stats(ap_server *s, ap_server_stats *out,
                              int reset_latencies);
ap_status ap_server_destroy(ap_server *s);

/*
 * ap_check_u32 -- check a sort's result on the device, the way the contest
 * program checked every result it timed (Sec. 1.1).  Adds into d_acc (three
 * uint64_t on the device, accumulated into, so zero them first):
 *   d_acc[0] += number of i < n-1 with d_keys[i] > d_keys[i+1] (unsigned)
 *   d_acc[1] += sum over the keys of SplitMix64(key), mod 2^64
 *   d_acc[2] ^= xor over the keys of SplitMix64(key)
 * An output is accepted when d_acc[0] is 0 and (d_acc[1], d_acc[2]) equal
 * those of its input: nondecreasing, and the same multiset of keys (the hash
 * does not depend on the order).  Reads each key once; nothing else written.
 */
ap_status ap_check_u32(const uint32_t *d_keys, size_t n, uint64_t *d_acc, void *stream);

/*
 * ap_check_u32_batch -- ap_check_u32 on `count` arrays in one launch
 * (0 <= count <= 65535): array a is d_keys[a] (a device pointer read from
 * device memory) with d_counts[a] keys, accumulated into d_acc[3a .. 3a+2].
 * max_n is an upper bound of the counts (it sizes the launch; a larger count
 * is still checked completely).  d_keys, d_counts and d_acc are 8-byte
 * aligned device arrays of count (d_acc: 3 * count) entries.  The launch has
 * count rows of min(ceil(max_n / 4096), 4 x CUs) workgroups, so batch arrays
 * of similar lengths: one 2^24-key array among 4095 short ones makes
 * 4096 x 1024 workgroups, most of which find no work (~20 ms).
 */
ap_status ap_check_u32_batch(const uint32_t *const *d_keys, const uint64_t *d_counts,
                             int count, size_t max_n, uint64_t *d_acc, void *stream);

/*
 * ap_release_cache -- free the scratch memory cached for ap_sort_u32,
 * ap_sort_pairs_u32 and the merge entry points on the current device (all
 * streams).  Synchronises the device first.  The segmented sort's per-stream
 * scratch and graphs, and a server's slots, are not affected.
 */
ap_status ap_release_cache(void);

/*
 * Kernel timing (tracing).  While enabled on the calling thread, every launch
 * made by a sort entry point of that thread is bracketed by two HIP events
 * recorded on the call's stream.  ap_profile_read waits for the recorded
 * events, adds each launch's duration to its kind, returns the totals and
 * clears them.  Kinds: AP_KIND_HIST (bucket counts + plan), AP_KIND_PASS + d
 * (digit pass d, d = 0..7; a pass the plan skips still records its near-empty
 * launch), AP_KIND_FINAL (copy + splitters), AP_KIND_MERGE (ap_merge_*), AP_KIND_SEG (segmented-sort
 * kernels).  ms and launches have at least AP_NKINDS entries.
 */
enum { AP_KIND_HIST = 0, AP_KIND_PASS = 1, AP_KIND_FINAL = 9, AP_KIND_SEG = 10, AP_KIND_MERGE = 11, AP_NKINDS = 16 };
ap_status ap_profile_enable(int on);
ap_status ap_profile_read(double *ms, uint64_t *launches, int nkinds);

/*
 * Rank primitive of every digit pass (single array, pairs, segmented and
 * served sorts).  The default rank gives each key the value returned by an
 * LDS atomic add on a per-wave bucket counter, which is stable because the LDS
 * services the conflicting lanes of one instruction in lane order; a device
 * self-check (run once per device by the first ap_sort_u32,
 * ap_sort_u32_segmented, ap_workspace_init or ap_server_create) confirms that
 * property before it is relied on.  Until then, or when it fails, the
 * alternative ranks run, which need no ordering property: per-bucket lane
 * masks in LDS (device-wide passes) and one ballot per digit bit (segmented
 * and served sorts).
 *
 * ap_rank_check_state: -1 = device not checked yet, 0 = check failed (the
 * order-agnostic ranks are used), 1 = check passed (the atomic rank is used).
 * ap_set_rank_mode: 0 = automatic (default), 1 = always the order-agnostic
 * ranks (process-wide; for testing both paths).
 */
int ap_rank_check_state(void);
ap_status ap_set_rank_mode(int mode);

/*
 * ap_debug_pass -- debug mode of the device-wide digit pass (Sec. 3.2 partial
 * sort and distribution of one digit), process-wide, for the keys-only passes
 * of ap_sort_u32, ap_sort_u32_ws, ap_sort_u32_noalloc and ap_sort_u32_msd.
 * The passes then run a separate kernel; the default kernels are not changed.
 *   mode 0: off (default).
 *   mode 1: timing perturbation.  Every tile sleeps, with probability 1/2 per
 *     point and for 0 - 12 us drawn from SplitMix64(seed, tile, digit, point),
 *     after its claim, before its scan, before its reorder, before the
 *     look-back, before publishing its inclusive prefix and before its scatter.
 *     Tiles then publish and finish in orders the normal timing seldom gives:
 *     a stress test of the look-back.  Results are unchanged (bit for bit).
 *   mode 2: phase trace.  d_trace (device memory, 8-byte aligned, holding
 *     trace_records records of 8 uint64) receives, for tile t of pass d of the
 *     last sort (record d * tiles + t; records beyond trace_records are not
 *     written), the wall clock (s_memrealtime, 100 MHz) when the tile was
 *     claimed, ranked, scanned, reordered, looked back and scattered (stores
 *     complete); words 6 and 7 are not written.  The trace kernel adds
 *     barriers after the rank and the reorder and waits for its stores, so a
 *     traced pass runs slightly slower.  d_trace must stay valid while sorts
 *     run in this mode.
 * Errors: AP_ERR_INVALID (mode outside 0..2; mode 2 without a buffer).
 */
ap_status ap_debug_pass(int mode, uint64_t seed, unsigned long long *d_trace, size_t trace_records);

/*
 * Tile shape of the device-wide digit pass (Sec. 3.2 partial sort and
 * distribution, one digit of the LSD sort of Sec. 3.3.1).  By default the
 * tile (one workgroup of 16 waves) grows with the array: 4K keys below 2^17,
 * 8K below 2^20, 16K below 2^22, 32K from there on (the mask rank uses 16K
 * where 32K is chosen; key-value pairs use at most 8K below 2^22 and 16K from
 * there on).
 * shape: -1 = by size (default), 0..3 = always 4K, 8K, 16K, 32K keys (pairs:
 * at most 16K).
 * Process-wide, for tests and tuning; results do not depend on it.  A
 * workspace sized by ap_sort_workspace_bytes before a change can be too small
 * afterwards (AP_ERR_INVALID).
 */
ap_status ap_set_pass_shape(int shape);

/* ap_last_error -- thread-local text for the last failure of this thread. */
const char *ap_last_error(void);

/* ap_version -- library version string. */
const char *ap_version(void);

#ifdef __cplusplus
}
#endif

#endif /* APSORT_H */
