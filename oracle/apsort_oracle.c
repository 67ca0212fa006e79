/*
 * CPU oracle for the radix sort of 32-bit integer keys (Weaver & Lynes,
 * "Sorting Integers on the AP1000").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library; it is plain, slow C (single-threaded, but for the timing
 * variant) written from the paper so that a reader can check it against the
 * text by eye.
 *
 * What it computes
 *   - oracle_digit_hist: the bucket histogram of one digit, the first loop of
 *     the bucket() procedure (Sec. 3.2): each element adds one to the count of
 *     its bucket.
 *   - oracle_bucket_pass: one such bucketing step on the 8-bit digit at a given
 *     shift, exposed so that tests can check single passes (their stability).
 *   - oracle_sort_u32: a least-significant-digit radix sort (Sec. 3.3.1): the
 *     keys are ordered by the lowest digit first and then by each higher digit
 *     in turn, each digit pass preserving the order left by the previous one.  Every
 *     pass is the bucketing step of Sec. 3.2 applied to one 8-bit digit: count
 *     the buckets, form cumulative totals (an exclusive prefix sum), then the
 *     partial sort that moves each element, in input order, to the next free
 *     slot of its bucket.  All four passes always run; nothing is skipped.
 *   - oracle_slice_starts / oracle_splitters: the output contract of Sec. 1.1
 *     (the sorted keys spread evenly over P cells, cell 0 holding the smallest)
 *     with the odd-count rule of the footnote in Sec. 3.4.2 (the cell with the
 *     lower id takes the extra element).  The splitter between cells p-1 and p
 *     is the first key of cell p; an empty cell gets the all-ones sentinel, in
 *     the spirit of the infinity padding of Sec. 2.1.1.
 *   - oracle_sort_segmented: the same sort applied independently to each
 *     segment [off[s], off[s+1]) of one array (one local sort per cell, the
 *     "Local Sort" phase of Sec. 3.3).
 *   - oracle_merge_u32: the merge step of the merge-exchange (Sec. 3.4: two
 *     sorted lists merged "in the classic manner"; Sec. 4.6: two sorted runs of
 *     one array merged): repeatedly move the smaller head element to the
 *     output, the first list's element on a tie.  Splitting the merged list at
 *     the first list's length gives the merge-exchange: the lower cell keeps
 *     the lower values, both cells keep their element counts.
 *   - oracle_sort_u32_mt: the same LSD sort with each pass split over T
 *     threads, for timing on a many-core host only.  Thread t takes the t-th
 *     contiguous chunk of the pass's input; the cumulative totals are taken
 *     over (bucket, thread) in that order, so thread t's elements of bucket v
 *     land after those of every lower bucket and after bucket v's elements of
 *     threads < t, and each thread moves its chunk in input order: the output
 *     of every pass is that of oracle_bucket_pass.
 *   - oracle_bucket_pass_pairs / oracle_sort_pairs_u32: the same bucketing
 *     pass and LSD sort with a 32-bit value travelling with every key.  Each
 *     pass keeps the order of elements with equal digits (Sec. 3.3.1), so
 *     pairs with equal keys leave in their input order: with values equal to
 *     input positions, the output values are the stable sorting permutation.
 *
 * Keys are unsigned 32-bit integers ordered as unsigned values (the paper sorts
 * positive integers; keys with bit 31 set are accepted as well).
 *
 * Error behaviour: functions return 0 on success and -1 when a scratch
 * allocation fails or an argument is invalid; nothing is written then.
 */
#define _POSIX_C_SOURCE 200809L
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_DIGIT_BITS 8
#define ORACLE_BUCKETS (1u << ORACLE_DIGIT_BITS)

/* Sec. 3.2, first loop of bucket(): one count per element added to the bucket
 * that its digit selects; the digit is the `bits`-bit field starting at bit
 * `shift`.  hist has 2^bits entries. */
int oracle_digit_hist(const uint32_t *keys, size_t n, int shift, int bits,
                      uint64_t *hist)
{
    if (bits < 1 || bits > 16 || shift < 0 || shift > 31 || (n && !keys) || !hist)
        return -1;
    size_t nb = (size_t)1 << bits;
    uint32_t mask = (uint32_t)(nb - 1);
    for (size_t v = 0; v < nb; ++v)
        hist[v] = 0;
    for (size_t i = 0; i < n; ++i)
        hist[(keys[i] >> shift) & mask] += 1;
    return 0;
}

/* One bucketing pass of Sec. 3.2 on the 8-bit digit at `shift`: bucket counts,
 * cumulative totals, then the partial sort, which leaves every bucket's
 * elements contiguous with the buckets in increasing order.  Elements are taken
 * in input order, so elements with equal digits keep their relative order. */
void oracle_bucket_pass(const uint32_t *src, uint32_t *dst, size_t n, int shift)
{
    uint64_t count[ORACLE_BUCKETS];
    uint64_t next[ORACLE_BUCKETS];
    for (unsigned v = 0; v < ORACLE_BUCKETS; ++v)
        count[v] = 0;
    for (size_t i = 0; i < n; ++i)
        count[(src[i] >> shift) & (ORACLE_BUCKETS - 1)] += 1;
    /* cumulative totals: first slot of each bucket */
    uint64_t running = 0;
    for (unsigned v = 0; v < ORACLE_BUCKETS; ++v) {
        next[v] = running;
        running += count[v];
    }
    /* partial sort */
    for (size_t i = 0; i < n; ++i) {
        unsigned v = (src[i] >> shift) & (ORACLE_BUCKETS - 1);
        dst[next[v]] = src[i];
        next[v] += 1;
    }
}

/* The bucketing pass above with a value moved together with each key: the
 * cumulative totals give the first slot of each bucket, then element j (in
 * input order) takes the next free slot of its bucket, its value with it. */
void oracle_bucket_pass_pairs(const uint32_t *src_k, const uint32_t *src_v,
                              uint32_t *dst_k, uint32_t *dst_v, size_t n, int shift)
{
    uint64_t first[ORACLE_BUCKETS];
    for (unsigned b = 0; b < ORACLE_BUCKETS; ++b)
        first[b] = 0;
    for (size_t j = 0; j < n; ++j)
        first[(src_k[j] >> shift) & (ORACLE_BUCKETS - 1)] += 1;
    uint64_t total = 0;
    for (unsigned b = 0; b < ORACLE_BUCKETS; ++b) {
        uint64_t c = first[b];
        first[b] = total;
        total += c;
    }
    for (size_t j = 0; j < n; ++j) {
        unsigned b = (src_k[j] >> shift) & (ORACLE_BUCKETS - 1);
        uint64_t slot = first[b]++;
        dst_k[slot] = src_k[j];
        dst_v[slot] = src_v[j];
    }
}

/* Sec. 3.3.1: LSD radix sort, low-order digit first, four 8-bit digits. */
int oracle_sort_u32(const uint32_t *in, uint32_t *out, size_t n)
{
    if (n == 0)
        return 0;
    if (!in || !out)
        return -1;
    uint32_t *a = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint32_t *b = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    memcpy(a, in, n * sizeof(uint32_t));
    for (int shift = 0; shift < 32; shift += ORACLE_DIGIT_BITS) {
        oracle_bucket_pass(a, b, n, shift);
        uint32_t *t = a;
        a = b;
        b = t;
    }
    memcpy(out, a, n * sizeof(uint32_t));
    free(a);
    free(b);
    return 0;
}

/* ---- timing variant: each bucketing pass split over threads ---- */
struct mt_job {
    const uint32_t *src;
    uint32_t *dst;
    size_t lo, hi;          /* this thread's chunk of the pass input */
    int shift;
    uint64_t *count;        /* ORACLE_BUCKETS counts of the chunk, then its first slots */
};

static void *mt_count(void *arg)
{
    struct mt_job *j = (struct mt_job *)arg;
    for (unsigned v = 0; v < ORACLE_BUCKETS; ++v)
        j->count[v] = 0;
    for (size_t i = j->lo; i < j->hi; ++i)
        j->count[(j->src[i] >> j->shift) & (ORACLE_BUCKETS - 1)] += 1;
    return NULL;
}

static void *mt_move(void *arg)
{
    struct mt_job *j = (struct mt_job *)arg;
    for (size_t i = j->lo; i < j->hi; ++i) {
        unsigned v = (j->src[i] >> j->shift) & (ORACLE_BUCKETS - 1);
        j->dst[j->count[v]] = j->src[i];
        j->count[v] += 1;
    }
    return NULL;
}

/* Runs fn on every job, one thread each (the calling thread takes job 0). */
static int mt_run(void *(*fn)(void *), struct mt_job *jobs, int nthreads, pthread_t *tid)
{
    int started = 0, rc = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tid[t], NULL, fn, &jobs[t]) != 0) {
            rc = -1;
            break;
        }
        started = t;
    }
    fn(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tid[t], NULL);
    if (rc != 0)                       /* finish the jobs no thread took */
        for (int t = started + 1; t < nthreads; ++t)
            fn(&jobs[t]);
    return 0;
}

int oracle_sort_u32_mt(const uint32_t *in, uint32_t *out, size_t n, int nthreads)
{
    if (n == 0)
        return 0;
    if (!in || !out || nthreads < 1 || nthreads > 1024)
        return -1;
    uint32_t *a = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint32_t *b = (uint32_t *)malloc(n * sizeof(uint32_t));
    struct mt_job *jobs = (struct mt_job *)malloc((size_t)nthreads * sizeof(struct mt_job));
    uint64_t *counts = (uint64_t *)malloc((size_t)nthreads * ORACLE_BUCKETS * sizeof(uint64_t));
    pthread_t *tid = (pthread_t *)malloc((size_t)nthreads * sizeof(pthread_t));
    if (!a || !b || !jobs || !counts || !tid) {
        free(a); free(b); free(jobs); free(counts); free(tid);
        return -1;
    }
    memcpy(a, in, n * sizeof(uint32_t));
    for (int pass = 0; pass * ORACLE_DIGIT_BITS < 32; ++pass) {
        const int shift = pass * ORACLE_DIGIT_BITS;
        for (int t = 0; t < nthreads; ++t) {
            jobs[t].src = a;
            jobs[t].dst = b;
            jobs[t].lo = n * (size_t)t / (size_t)nthreads;
            jobs[t].hi = n * (size_t)(t + 1) / (size_t)nthreads;
            jobs[t].shift = shift;
            jobs[t].count = counts + (size_t)t * ORACLE_BUCKETS;
        }
        mt_run(mt_count, jobs, nthreads, tid);
        /* cumulative totals over (bucket, thread): first slot of thread t's part of bucket v */
        uint64_t running = 0;
        for (unsigned v = 0; v < ORACLE_BUCKETS; ++v)
            for (int t = 0; t < nthreads; ++t) {
                uint64_t c = jobs[t].count[v];
                jobs[t].count[v] = running;
                running += c;
            }
        mt_run(mt_move, jobs, nthreads, tid);
        uint32_t *t = a;
        a = b;
        b = t;
    }
    memcpy(out, a, n * sizeof(uint32_t));
    free(a); free(b); free(jobs); free(counts); free(tid);
    return 0;
}

/* Sec. 3.3.1 for (key, value) pairs: four stable bucketing passes on the
 * keys' 8-bit digits, low digit first, every value moving with its key. */
int oracle_sort_pairs_u32(const uint32_t *in_k, const uint32_t *in_v,
                          uint32_t *out_k, uint32_t *out_v, size_t n)
{
    if (n == 0)
        return 0;
    if (!in_k || !in_v || !out_k || !out_v)
        return -1;
    uint32_t *buf = (uint32_t *)malloc(4 * n * sizeof(uint32_t));
    if (!buf)
        return -1;
    /* two (keys, values) buffers; pass d reads buffer d % 2 and writes the other */
    uint32_t *keys[2] = {buf, buf + 2 * n};
    uint32_t *vals[2] = {buf + n, buf + 3 * n};
    memcpy(keys[0], in_k, n * sizeof(uint32_t));
    memcpy(vals[0], in_v, n * sizeof(uint32_t));
    for (int d = 0; d < 4; ++d)
        oracle_bucket_pass_pairs(keys[d % 2], vals[d % 2], keys[(d + 1) % 2], vals[(d + 1) % 2], n,
                                 d * ORACLE_DIGIT_BITS);
    memcpy(out_k, keys[0], n * sizeof(uint32_t));  /* after four passes: buffer 0 */
    memcpy(out_v, vals[0], n * sizeof(uint32_t));
    free(buf);
    return 0;
}

/* Sec. 3.4 / 4.6: merge of two nondecreasing lists; ties take the first list's
 * element first.  out must not overlap a or b. */
int oracle_merge_u32(const uint32_t *a, size_t na, const uint32_t *b, size_t nb, uint32_t *out)
{
    if ((na && !a) || (nb && !b) || ((na + nb) && !out))
        return -1;
    size_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) {
        if (b[j] < a[i])
            out[k++] = b[j++];
        else
            out[k++] = a[i++];
    }
    while (i < na)
        out[k++] = a[i++];
    while (j < nb)
        out[k++] = b[j++];
    return 0;
}

/* Sec. 1.1 with the footnote of Sec. 3.4.2: cell p of P holds the sorted
 * positions [starts[p], starts[p+1]); the first n mod P cells hold one extra
 * element.  starts has P+1 entries. */
int oracle_slice_starts(size_t n, int P, uint64_t *starts)
{
    if (P < 1 || !starts)
        return -1;
    uint64_t q = n / (uint64_t)P, r = n % (uint64_t)P;
    uint64_t pos = 0;
    for (int p = 0; p < P; ++p) {
        starts[p] = pos;
        pos += q + ((uint64_t)p < r ? 1 : 0);
    }
    starts[P] = pos;
    return 0;
}

/* Splitter p-1 (p = 1..P-1) is the lowest key held by cell p, or the
 * all-ones sentinel (infinity padding, Sec. 2.1.1) when cell p is empty. */
int oracle_splitters(const uint32_t *sorted, size_t n, int P, uint32_t *splitters)
{
    if (P < 1 || (n && !sorted) || (P > 1 && !splitters))
        return -1;
    uint64_t *starts = (uint64_t *)malloc(((size_t)P + 1) * sizeof(uint64_t));
    if (!starts)
        return -1;
    oracle_slice_starts(n, P, starts);
    for (int p = 1; p < P; ++p)
        splitters[p - 1] = (starts[p] < starts[p + 1]) ? sorted[starts[p]] : 0xFFFFFFFFu;
    free(starts);
    return 0;
}

/* Sec. 3.3: one independent local sort per segment [off[s], off[s+1]). */
int oracle_sort_segmented(uint32_t *keys, const uint64_t *offsets, int nseg)
{
    if (nseg < 0 || (nseg > 0 && (!offsets || !keys)))
        return -1;
    for (int s = 0; s < nseg; ++s)
        if (offsets[s + 1] < offsets[s])
            return -1;
    for (int s = 0; s < nseg; ++s) {
        size_t len = (size_t)(offsets[s + 1] - offsets[s]);
        if (oracle_sort_u32(keys + offsets[s], keys + offsets[s], len) != 0)
            return -1;
    }
    return 0;
}
