#!/usr/bin/env python3
"""Benchmark of the radix sort on one MI355X.  Prints ONE JSON line.

Main metric: a step is one full sort (bucket counts + plan, every digit pass, splitters) of 2^26
uint32 keys, i.i.d. uniform in [0, 2^31-1] (distribution (a), seed 1), already resident in HBM,
into P = 64 cells; `value` is keys sorted per second over the K timed steps (Gkeys/s).

`roofline` describes the digit-pass kernel k_pass: algorithmic bytes per launch (8 B per key) over
the mean launch duration, timed with HIP events recorded around each launch on the sort's stream
(in a second loop of the same sorts right after the timed steps: the events cost time of their
own).  `traffic` and the rocprofv3 mean duration come from the committed profile summary when it
was taken on the current kernel source.

Extra fields (each can be skipped): the other distributions (b)-(e) at 2^26 and the adversarial
2^27 set; the per-pass roofline at 2^27 uniform keys (twice the size of the 256 MB memory-side
cache); the 4096-segment batch (lengths log-uniform in [64, 2^18]) sorted by the batched segmented
form vs a loop of plain per-array launches; the served form: 100k requests (Poisson arrivals,
log-uniform [2^10, 2^24] keys) at swept rates vs one plain launch per request, FIFO on one stream,
every output checked on the device (order + multiset hash) and a seeded 1% sample against the
oracle; p50/p99 latency of a 2^20-key sort.  The CPU baseline is the oracle (plain C LSD radix
sort) on the same 2^26 keys, single-threaded and with every pass split over the host's threads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gkeys/s on 64M u32 & 4096-segment batch; % HBM roofline; p50/p99 ms"
HBM_PEAK_GBS = 8000.0
N_MAIN = 1 << 26
# the pass kernel, its tile core and the device helpers it inlines (rank, look-back words)
KERNEL_SRCS = [os.path.join(ROOT, "paper_cs_0004013_amd", "csrc", f)
               for f in ("apsort_kernels.h", "apsort_pass_core.h", "apsort_device.h")]
COUNTERS = os.path.join(ROOT, "profiles", "k_pass_counters_uniform_2p26.md")


def kernel_sha() -> str:
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SRCS)).hexdigest()[:16]


def read_profile() -> dict | None:
    """HBM bytes and mean duration per k_pass launch from the committed rocprofv3 summary, or None
    when the summary is missing or was taken on a different kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    vals = {}
    for line in open(COUNTERS):
        line = line.strip().strip("|").strip()
        if ":" in line and not line.startswith("#"):
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_sha():
        return None
    try:
        return {"traffic": float(vals["hbm_bytes_per_launch"]), "mean_us": float(vals["mean_duration_us"])}
    except (KeyError, ValueError):
        return None


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_sorts(binding, torch, t_in, t_out, spl, steps: int, warmup: int, profile: bool):
    for _ in range(warmup):
        binding.ap_sort_u32(t_in, t_out, 64, spl)
    torch.cuda.synchronize()
    if profile:
        binding.ap_profile_read()           # drop warm-up records
        binding.ap_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        binding.ap_sort_u32(t_in, t_out, 64, spl)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if profile:
        binding.ap_profile_enable(False)
        prof = binding.ap_profile_read()
    return dt, prof


def pass_stats(binding, prof):
    """Mean duration (s) of the digit-pass launches that ran, from HIP-event records."""
    ms, launches = prof
    pass_ms = sum(ms[binding.AP_KIND_PASS + d] for d in range(4))
    n = sum(launches[binding.AP_KIND_PASS + d] for d in range(4))
    return pass_ms / max(n, 1) / 1e3


def pct(v, p):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), p)) if len(v) else None


# ------------------------------------------------------------------------------------------------
def sort_latency(binding, torch, np, keys):
    """p50/p99 latency of ap_sort_u32 (64 cells) over 50 timed sorts after 5 warm-ups."""
    t_in = torch.from_numpy(keys.view(np.int32)).to("cuda")
    t_out = torch.empty_like(t_in)
    spl = torch.empty(63, dtype=torch.int32, device="cuda")
    ms = []
    for i in range(55):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        binding.ap_sort_u32(t_in, t_out, 64, spl)
        b.record()
        torch.cuda.synchronize()
        if i >= 5:
            ms.append(a.elapsed_time(b))
    n = int(keys.size)
    return {"n": n, "p50_ms": round(pct(ms, 50), 4), "p99_ms": round(pct(ms, 99), 4),
            "gkeys_s_p50": round(n / pct(ms, 50) / 1e6, 2)}


def leg_latency(binding, torch, np, inputs):
    """2^20 uniform keys (seed 0), 64 cells: per-sort latency; also 2^12 and 2^14 keys, which take
    the one-workgroup path."""
    res = sort_latency(binding, torch, np, inputs.keyset("a", 1 << 20, seed=0).keys)
    res["small"] = [sort_latency(binding, torch, np, inputs.keyset("a", n, seed=0).keys) for n in (1 << 12, 1 << 14)]
    return res


def leg_pass_2p27(binding, torch, np, inputs, spl):
    """Per-pass roofline at 2^27 uniform keys (seed 7): 1 GiB of keys per pass, four times the
    memory-side cache, so no pass can be served from it."""
    n = 1 << 27
    t_in = torch.from_numpy(inputs.keyset("a", n, seed=7).keys.view(np.int32)).to("cuda")
    t_out = torch.empty_like(t_in)
    dt, _ = time_sorts(binding, torch, t_in, t_out, spl, 10, 3, False)
    _, prof = time_sorts(binding, torch, t_in, t_out, spl, 10, 1, True)
    pass_s = pass_stats(binding, prof)
    gbs = 8 * n / pass_s / 1e9
    return {"n": n, "ms_per_sort": round(dt * 1e3 / 10, 4), "gkeys_s": round(n * 10 / dt / 1e9, 3),
            "pass_us": round(pass_s * 1e6, 2), "pass_gbs": round(gbs, 1),
            "pass_frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4)}


def leg_msd(binding, torch, np, pools, spl, steps: int = 10):
    """The bucketing variant (top 16 bits, then a local sort per bucket) against the LSD sort on
    the same 2^26 keys, distributions (a) and (e); outputs compared with the LSD sort's."""
    res = {}
    for dist in ("a", "e"):
        if dist not in pools:
            continue
        t_in = pools[dist]
        n = t_in.numel()
        out_m, out_l = torch.empty_like(t_in), torch.empty_like(t_in)
        times = {}
        for name, fn, out in (("msd", binding.ap_sort_u32_msd, out_m), ("lsd", binding.ap_sort_u32, out_l)):
            for _ in range(3):
                fn(t_in, out, 64, spl)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                fn(t_in, out, 64, spl)
            e1.record()
            torch.cuda.synchronize()
            times[name] = e0.elapsed_time(e1) / steps
        res[dist] = {"msd_ms": round(times["msd"], 4), "msd_gkeys_s": round(n / times["msd"] / 1e6, 3),
                     "lsd_ms": round(times["lsd"], 4), "lsd_gkeys_s": round(n / times["lsd"] / 1e6, 3),
                     "same_output": bool(torch.equal(out_m, out_l))}
    return res


def leg_pairs(binding, torch, np, inputs, t_keys, steps: int = 10):
    """(key, value) pairs: the same 2^26 uniform keys with values 0..n-1 (an argsort); per-pass
    time from HIP events, 16 algorithmic bytes per key per pass (key and value, read and write)."""
    n = t_keys.numel()
    vals = torch.arange(n, dtype=torch.int32, device="cuda")
    k_out = torch.empty_like(t_keys)
    v_out = torch.empty_like(vals)
    for _ in range(3):
        binding.ap_sort_pairs_u32(t_keys, vals, k_out, v_out, 64, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        binding.ap_sort_pairs_u32(t_keys, vals, k_out, v_out, 64, None)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    binding.ap_profile_read()
    binding.ap_profile_enable(True)
    for _ in range(steps):
        binding.ap_sort_pairs_u32(t_keys, vals, k_out, v_out, 64, None)
    torch.cuda.synchronize()
    binding.ap_profile_enable(False)
    pass_us = pass_stats(binding, binding.ap_profile_read()) * 1e6
    return {"n": n, "ms_per_sort": round(dt * 1e3, 4), "gpairs_s": round(n / dt / 1e9, 3),
            "pass_us": round(pass_us, 2), "pass_gbs": round(16 * n / pass_us / 1e3, 1),
            "pass_frac_of_8tbs": round(16 * n / pass_us / 1e3 / HBM_PEAK_GBS, 4)}


def leg_merge(binding, torch, np, inputs, t_keys, steps: int = 10):
    """Merge of two sorted runs of 2^25 keys each (the sorted halves of the 2^26 uniform keys):
    8 algorithmic bytes per output key (read once, written once)."""
    n = t_keys.numel()
    a = torch.sort(t_keys[: n // 2])[0]
    b = torch.sort(t_keys[n // 2:])[0]
    out = torch.empty_like(t_keys)
    for _ in range(3):
        binding.ap_merge_u32(a, b, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        binding.ap_merge_u32(a, b, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ok = bool(torch.equal(out, torch.sort(t_keys)[0]))
    return {"n": n, "ms": round(ms, 4), "gkeys_s": round(n / ms / 1e6, 2), "gbs": round(8 * n / ms / 1e6, 1),
            "frac_of_8tbs": round(8 * n / ms / 1e6 / HBM_PEAK_GBS, 4), "ok": ok}


def check_arrays(binding, torch, np, base_ptr: int, offsets, stream=None):
    """Device check of the arrays [offsets[s], offsets[s+1]) of the int32 buffer at base_ptr:
    (descents, SplitMix64 sum, xor) per array, as a (nseg, 3) uint64 numpy array."""
    off = np.asarray(offsets, dtype=np.int64)
    lens = np.diff(off)
    out = np.zeros((lens.size, 3), dtype=np.uint64)
    # A batched check launches (arrays x blocks for its longest array) workgroups: arrays of more
    # than 2^20 keys are checked one per call, the rest in batches sized by the longest of them.
    big = lens > (1 << 20)
    for sel in (np.nonzero(big)[0], np.nonzero(~big)[0]):
        if sel.size == 0:
            continue
        ptrs = torch.from_numpy(base_ptr + 4 * off[sel]).to("cuda")
        cnts = torch.from_numpy(lens[sel]).to("cuda")
        acc = torch.zeros((sel.size, 3), dtype=torch.int64, device="cuda")
        step = 1 if big[sel[0]] else 4096
        for s0 in range(0, sel.size, step):
            c = min(step, sel.size - s0)
            binding.ap_check_u32_batch(ptrs.data_ptr() + 8 * s0, cnts.data_ptr() + 8 * s0, c,
                                       int(lens[sel[s0:s0 + c]].max()), acc.data_ptr() + 24 * s0, stream)
        torch.cuda.synchronize()
        out[sel] = acc.cpu().numpy().view(np.uint64)
    return out


def leg_segmented(binding, torch, np, inputs, steps: int, baseline: bool = True):
    """4096 segments, lengths log-uniform in [64, 2^18] (seed 0); segment s uses seed s.  Every
    segment of the result is checked on the device: no descent, and the SplitMix64 multiset hash
    of the segment's input."""
    L = inputs.segment_lengths(4096, seed=0)
    keys, off, _ = inputs.segment_keys(L)
    n = int(keys.size)
    s = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(s):
        t_src = torch.from_numpy(keys.view(np.int32)).to("cuda")
        t_work = torch.empty_like(t_src)
        t_off = torch.from_numpy(off.view(np.int32)).to("cuda")
        ms = []
        for i in range(steps + 2):
            t_work.copy_(t_src)              # restore the unsorted input (outside the timed region)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            binding.ap_sort_u32_segmented(t_work, t_off, stream=s)
            b.record(s)
            s.synchronize()
            if i >= 2:
                ms.append(a.elapsed_time(b))
        h_in = check_arrays(binding, torch, np, t_src.data_ptr(), off)
        h_out = check_arrays(binding, torch, np, t_work.data_ptr(), off)
        bad = int(np.count_nonzero((h_out[:, 0] != 0) | np.any(h_out[:, 1:] != h_in[:, 1:], axis=1)))
        res["segments"] = 4096
        res["keys"] = n
        res["batched_ms_p50"] = round(pct(ms, 50), 4)
        res["batched_gkeys_s"] = round(n / pct(ms, 50) / 1e6, 3)
        res["segments_bad"] = bad
        res["batched_ok"] = bad == 0
        if not baseline:
            return res
        # baseline: one plain ap_sort_u32 per segment, in order, on the same stream
        lib = binding.lib()
        base_ptr = t_work.data_ptr()
        offs = off.astype(np.int64)
        sid = s.cuda_stream
        ms_b = []
        for i in range(2):
            t_work.copy_(t_src)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            for k in range(4096):
                p = base_ptr + 4 * int(offs[k])
                st = lib.ap_sort_u32(p, p, int(offs[k + 1] - offs[k]), 1, None, sid)
                if st:
                    raise RuntimeError(f"ap_sort_u32 failed: {binding.last_error()}")
            b.record(s)
            s.synchronize()
            ms_b.append(a.elapsed_time(b))
        res["loop_of_plain_launches_ms"] = round(min(ms_b), 3)
        res["loop_of_plain_launches_gkeys_s"] = round(n / min(ms_b) / 1e6, 3)
        res["speedup_vs_loop"] = round(min(ms_b) / pct(ms, 50), 2)
    return res


def leg_segmented_long(binding, torch, np, inputs, spl, steps: int = 5):
    """Long segments through the device-wide passes: (i) 4 segments of 2^24 uniform keys among
    4092 log-uniform short ones ([64, 2^14], seed 3), (ii) one segment of 2^28 uniform keys; each
    against ap_sort_u32 of the same keys as one array.  Checked on the device per segment."""
    rng = np.random.default_rng(5)
    short = inputs.segment_lengths(4092, seed=3, lo=64, hi=1 << 14)
    L = np.concatenate([[1 << 24] * 4, short]).astype(np.int64)
    L = L[rng.permutation(L.size)]
    off_a = np.zeros(L.size + 1, np.int64)
    np.cumsum(L, out=off_a[1:])
    res = {"long_min": binding.ap_segmented_get_long_min()}
    cases = [("four_2p24_plus_4092_short", inputs.keyset("a", int(off_a[-1]), seed=11).keys, off_a),
             ("one_2p28", inputs.keyset("a", 1 << 28, seed=12).keys, np.array([0, 1 << 28], np.int64))]
    s = torch.cuda.Stream()
    for name, keys, off in cases:
        n = int(keys.size)
        with torch.cuda.stream(s):
            t_src = torch.from_numpy(keys.view(np.int32)).to("cuda")
            t_work = torch.empty_like(t_src)
            t_off = torch.from_numpy(off.astype(np.uint32).view(np.int32)).to("cuda")
            ms = []
            for i in range(steps + 2):
                t_work.copy_(t_src)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(s)
                binding.ap_sort_u32_segmented(t_work, t_off, stream=s)
                b.record(s)
                s.synchronize()
                if i >= 2:
                    ms.append(a.elapsed_time(b))
            h_in = check_arrays(binding, torch, np, t_src.data_ptr(), off)
            h_out = check_arrays(binding, torch, np, t_work.data_ptr(), off)
            bad = int(np.count_nonzero((h_out[:, 0] != 0) | np.any(h_out[:, 1:] != h_in[:, 1:], axis=1)))
            t_out = torch.empty_like(t_src)
            for _ in range(2):
                binding.ap_sort_u32(t_src, t_out, 1, None, stream=s)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(steps):
                binding.ap_sort_u32(t_src, t_out, 1, None, stream=s)
            e1.record(s)
            s.synchronize()
            plain = e0.elapsed_time(e1) / steps
            seg = pct(ms, 50)
            res[name] = {"keys": n, "segments": int(off.size - 1), "segmented_ms_p50": round(seg, 4),
                         "segmented_gkeys_s": round(n / seg / 1e6, 3), "plain_sort_ms": round(plain, 4),
                         "plain_sort_gkeys_s": round(n / plain / 1e6, 3), "ratio": round(plain / seg, 3),
                         "segments_bad": bad}
            del t_src, t_work, t_out
    return res


# ------------------------------------------------------------------------------------------------
def phase_trace(binding, torch, np, inputs, sorts: int = 5) -> str:
    """Per-tile phase timestamps of the digit passes of a 2^26 uniform sort (the traced kernel,
    ap_debug_pass mode 2, which adds two barriers and a wait for its stores), as a markdown
    summary: duration of each phase per tile, and the mean number of tiles in flight."""
    n = N_MAIN
    t_in = torch.from_numpy(inputs.keyset("a", n, seed=1).keys.view(np.int32)).to("cuda")
    t_out = torch.empty_like(t_in)
    tile = 16 * 64 * 32
    ntiles = (n + tile - 1) // tile
    W = binding.PASS_TRACE_WORDS
    trace = torch.zeros(4 * ntiles * W, dtype=torch.int64, device="cuda")
    binding.ap_debug_pass(binding.PASS_DBG_TRACE, 0, trace)
    try:
        for _ in range(sorts):
            binding.ap_sort_u32(t_in, t_out, 64, None)
        torch.cuda.synchronize()
    finally:
        binding.ap_debug_pass(binding.PASS_DBG_NONE)
    ok = bool(torch.equal(t_out, torch.sort(t_in)[0]))
    rec = trace.cpu().numpy().reshape(4, ntiles, W)[:, :, :6].astype(np.float64) / 100.0  # 100 MHz -> us
    names = ["claim to rank done (loads + rank)", "scan of the tile's counts", "publish + LDS reorder",
             "look-back", "scatter (stores complete)"]
    lines = ["# k_pass phase timestamps, 2^26 uniform 31-bit keys (dist a, seed 1), 32K-key tiles", "",
             "Command (run from the repository root on an MI355X):", "", "```",
             "python3 bench.py --phase-trace > profiles/k_pass_phases_uniform_2p26.md", "```", "",
             f"The last of {sorts} sorts; traced kernel (ap_debug_pass mode 2: per-tile s_memrealtime stamps by "
             "thread 0, with a barrier after the rank and after the reorder and a wait for the scatter's stores). "
             f"Output sorted: {ok}.", "",
             "| phase | mean us | p50 us | p90 us |", "|---|---|---|---|"]
    for i, nm in enumerate(names):
        dur = (rec[:, :, i + 1] - rec[:, :, i]).ravel()
        lines.append(f"| {nm} | {dur.mean():.2f} | {np.percentile(dur, 50):.2f} | {np.percentile(dur, 90):.2f} |")
    tot = (rec[:, :, 5] - rec[:, :, 0]).ravel()
    lines.append(f"| whole tile | {tot.mean():.2f} | {np.percentile(tot, 50):.2f} | {np.percentile(tot, 90):.2f} |")
    lines += ["", "| pass | wall us (first claim to last scatter) | mean tiles in flight |", "|---|---|---|"]
    for d in range(4):
        wall = rec[d, :, 5].max() - rec[d, :, 0].min()
        busy = (rec[d, :, 5] - rec[d, :, 0]).sum()
        lines.append(f"| {d} | {wall:.1f} | {busy / wall:.1f} |")
    return "\n".join(lines) + "\n"


# ------------------------------------------------------------------------------------------------
class ServedTrace:
    """The served workload: nreq requests, request r drawing its size (log-uniform [2^10, 2^24]),
    distribution and window into that distribution's device-resident pool from seed r.  Sizes,
    windows and inputs do not depend on the arrival rate, so the input hashes and the oracle's
    results for the seeded 1% sample are computed once and serve every rate point."""

    RING = 256            # output buffers of 2^24 keys, reused round-robin
    CAP = 1 << 24
    BATCH = 64            # outputs checked per device check launch

    def __init__(self, binding, torch, np, inputs, pools_dev, pools_host, nreq: int):
        import oracle
        self.b, self.torch, self.np, self.inputs = binding, torch, np, inputs
        self.nreq = nreq
        self.pool_keys = int(next(iter(pools_dev.values())).numel())
        self.tr = inputs.request_trace(nreq, rate_per_s=1.0, pool_keys=self.pool_keys, seed=0)
        self.n = np.array([r.n for r in self.tr], dtype=np.int64)
        self.total_keys = int(self.n.sum())
        self.ring = torch.empty(self.RING * self.CAP, dtype=torch.int32, device="cuda")
        self.spl_ring = torch.empty(self.RING * 64, dtype=torch.int32, device="cuda")
        slot = np.arange(nreq) % self.RING
        self.src = np.array([pools_dev[r.dist].data_ptr() + 4 * r.pool_offset for r in self.tr], dtype=np.int64)
        self.out = self.ring.data_ptr() + 4 * self.CAP * slot
        self.spl = self.spl_ring.data_ptr() + 4 * 64 * slot
        self.d_out = torch.from_numpy(self.out).to("cuda")
        self.d_n = torch.from_numpy(self.n).to("cuda")
        nb = (nreq + self.BATCH - 1) // self.BATCH
        self.batch_max = np.array([self.n[k * self.BATCH:(k + 1) * self.BATCH].max() for k in range(nb)])
        d_src = torch.from_numpy(self.src).to("cuda")
        self.acc_in = torch.zeros((nreq, 3), dtype=torch.int64, device="cuda")
        for j0 in range(0, nreq, 4096):
            c = min(4096, nreq - j0)
            binding.ap_check_u32_batch(d_src.data_ptr() + 8 * j0, self.d_n.data_ptr() + 8 * j0, c,
                                       int(self.n[j0:j0 + c].max()), self.acc_in.data_ptr() + 24 * j0)
        # seeded 1% sample: expected outputs and splitters from the oracle (its timing variant,
        # pinned bit-exact to the single-thread oracle), kept on the device
        self.sample = np.sort(inputs.rng_for(4242).choice(nreq, max(1, nreq // 100), replace=False))
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        exp_off = np.zeros(self.sample.size + 1, dtype=np.int64)
        np.cumsum(self.n[self.sample], out=exp_off[1:])
        exp = np.empty(int(exp_off[-1]), dtype=np.uint32)
        exp_spl = np.empty((self.sample.size, 63), dtype=np.uint32)
        for k, r in enumerate(self.sample):
            q = self.tr[r]
            w = oracle.sort_u32_mt(pools_host[q.dist][q.pool_offset:q.pool_offset + q.n], threads)
            exp[exp_off[k]:exp_off[k + 1]] = w
            exp_spl[k] = oracle.splitters(w, 64)
        self.exp = torch.from_numpy(exp.view(np.int32)).to("cuda")
        self.exp_spl = torch.from_numpy(exp_spl.view(np.int32)).to("cuda")
        self.exp_off = exp_off
        self.sample_pos = {int(r): k for k, r in enumerate(self.sample)}
        self.sample_keys = int(exp_off[-1])

    def arrivals(self, rate: float):
        tr = self.inputs.request_trace(self.nreq, rate_per_s=rate, pool_keys=self.pool_keys, seed=0)
        return self.np.array([r.arrival_s for r in tr], dtype=self.np.float64)

    def check_batch(self, k: int, acc, mism, stream):
        """Device check of the outputs of requests [k*BATCH, (k+1)*BATCH) on `stream`, and the
        bit-exact comparison of the sampled ones with the oracle's outputs."""
        torch = self.torch
        j0, j1 = k * self.BATCH, min((k + 1) * self.BATCH, self.nreq)
        # max_n sizes the launch (workgroups per array): the batch's own longest request
        self.b.ap_check_u32_batch(self.d_out.data_ptr() + 8 * j0, self.d_n.data_ptr() + 8 * j0, j1 - j0,
                                  int(self.batch_max[k]), acc.data_ptr() + 24 * j0, stream)
        hits = [j for j in range(j0, j1) if j in self.sample_pos]
        if hits:
            with torch.cuda.stream(stream):
                for j in hits:
                    s, n = self.sample_pos[j], int(self.n[j])
                    b = j % self.RING
                    got = self.ring[b * self.CAP: b * self.CAP + n]
                    mism[0] += (got != self.exp[self.exp_off[s]:self.exp_off[s] + n]).sum()
                    mism[1] += (self.spl_ring[b * 64: b * 64 + 63] != self.exp_spl[s]).sum()

    def verdict(self, acc, mism) -> dict:
        np = self.np
        a = acc.cpu().numpy().view(np.uint64)
        h = self.acc_in.cpu().numpy().view(np.uint64)
        bad = int(np.count_nonzero((a[:, 0] != 0) | np.any(a[:, 1:] != h[:, 1:], axis=1)))
        m = mism.cpu().numpy()
        return {"outputs_checked": self.nreq, "outputs_bad": bad, "sample_checked": int(self.sample.size),
                "sample_keys": self.sample_keys, "sample_keys_bad": int(m[0]), "sample_splitters_bad": int(m[1])}


def run_served(st: ServedTrace, srv, arr_s) -> dict:
    """Open loop: request i is submitted at its arrival time with its arrival timestamp (the
    server measures latency from it); the outputs of whole batches of requests are checked on a
    side stream RING/2 requests behind, and an output buffer is reused only after its check."""
    torch, np = st.torch, st.np
    R, B = st.RING, st.BATCH
    acc = torch.zeros((st.nreq, 3), dtype=torch.int64, device="cuda")
    mism = torch.zeros(2, dtype=torch.int64, device="cuda")
    V = torch.cuda.Stream()
    nev = R // B + 3
    evs = [torch.cuda.Event() for _ in range(nev)]
    tickets = [0] * st.nreq
    lag = np.zeros(st.nreq)
    st0 = srv.stats(reset_latencies=True)
    t0 = time.monotonic_ns() + 2_000_000
    arr = t0 + (arr_s * 1e9).astype(np.int64)
    synced = 0                                   # check batches known complete: [0, synced)
    retired = 0                                  # check batches launched: [0, retired)

    def retire(k):
        for j in range(k * B, min((k + 1) * B, st.nreq)):
            s_ = srv.wait(tickets[j])
            if s_:
                raise RuntimeError(f"served request {j} failed with status {s_}")
        st.check_batch(k, acc, mism, V)
        evs[k % nev].record(V)

    src, out, spl, n = st.src, st.out, st.spl, st.n
    for i in range(st.nreq):
        a = int(arr[i])
        while time.monotonic_ns() < a:
            pass
        if i >= R:
            need = (i - R) // B + 1
            while synced < need:
                evs[synced % nev].synchronize()
                synced += 1
        tickets[i] = srv.submit_at_ptr(int(src[i]), int(out[i]), int(n[i]), 64, int(spl[i]), a)
        lag[i] = time.monotonic_ns() - a
        while (retired + 1) * B <= i + 1 - R // 2:
            retire(retired)
            retired += 1
    while retired * B < st.nreq:
        retire(retired)
        retired += 1
    V.synchronize()
    wall = (time.monotonic_ns() - t0) / 1e9
    stt = srv.stats(reset_latencies=True)
    return {"gkeys_s": round(st.total_keys / wall / 1e9, 3), "p50_ms": round(stt["p50_us"] / 1e3, 4),
            "p99_ms": round(stt["p99_us"] / 1e3, 4), "latency_from": "arrival",
            "queue_p50_ms": round(stt["queue_p50_us"] / 1e3, 4), "queue_p99_ms": round(stt["queue_p99_us"] / 1e3, 4),
            "scratch_peak_gib": round(stt["scratch_peak_bytes"] / 2**30, 3),
            "submit_lag_mean_ms": round(float(lag.mean()) / 1e6, 4),
            "submit_lag_max_ms": round(float(lag.max()) / 1e6, 3),
            "batches": stt["batches"] - st0["batches"], "alone": stt["alone"] - st0["alone"],
            **st.verdict(acc, mism)}


def run_plain(st: ServedTrace, arr_s, closed_loop: bool = False) -> dict:
    """One plain ap_sort_u32 per request, FIFO on one stream, launched at its arrival time (or
    back to back).  Latency = completion - arrival on the host clock, as the server measures it:
    the loop polls the requests' completion events in order while it waits for the next arrival
    (and once after each launch), and stamps each completion when it sees it.  The latency from
    GPU event times (completion event - a start event recorded at t0) is kept beside it; it reads
    lower, since it starts the clock when the GPU processes the start event, not at t0.  The same
    device checks run on the stream after every BATCH requests."""
    torch, np = st.torch, st.np
    lib = st.b.lib()
    B = st.BATCH
    acc = torch.zeros((st.nreq, 3), dtype=torch.int64, device="cuda")
    mism = torch.zeros(2, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(st.nreq)]
    start = torch.cuda.Event(enable_timing=True)
    sid = s.cuda_stream
    src, out, spl, n = st.src, st.out, st.spl, st.n
    done_ns = np.zeros(st.nreq, dtype=np.int64)
    seen = 0  # completions stamped: [0, seen)

    def poll(launched):
        nonlocal seen
        while seen < launched and evs[seen].query():
            done_ns[seen] = time.monotonic_ns()
            seen += 1

    arr_ns = None if closed_loop else (np.asarray(arr_s, dtype=np.float64) * 1e9).astype(np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t0_ns = time.monotonic_ns()
    start.record(s)
    for i in range(st.nreq):
        if not closed_loop:
            a = t0_ns + int(arr_ns[i])
            while time.monotonic_ns() < a:
                poll(i)
        r = lib.ap_sort_u32(int(src[i]), int(out[i]), int(n[i]), 64, int(spl[i]), sid)
        if r:
            raise RuntimeError(st.b.last_error())
        evs[i].record(s)
        if not closed_loop:
            poll(i + 1)
        if (i + 1) % B == 0 or i + 1 == st.nreq:
            st.check_batch(i // B, acc, mism, s)
    if not closed_loop:
        while seen < st.nreq:
            poll(st.nreq)
    s.synchronize()
    wall = time.perf_counter() - t0
    res = {"gkeys_s": round(st.total_keys / wall / 1e9, 3), "req_s": round(st.nreq / wall, 1)}
    if not closed_loop:
        lat = (done_ns - t0_ns - arr_ns) / 1e6
        lat_ev = [start.elapsed_time(evs[i]) - float(arr_s[i]) * 1e3 for i in range(st.nreq)]
        res.update({"p50_ms": round(pct(lat, 50), 4), "p99_ms": round(pct(lat, 99), 4), "latency_from": "arrival",
                    "p50_ms_gpu_events": round(pct(lat_ev, 50), 4), "p99_ms_gpu_events": round(pct(lat_ev, 99), 4)})
    res.update(st.verdict(acc, mism))
    return res


def leg_served(binding, torch, np, inputs, pools_dev, pools_host, nreq: int, rates, rates_small,
               alone_min_keys: int = 1 << 16):
    """The served form against one plain launch per request, at offered rates that are fractions of
    the plain form's measured capacity; the server with a 64 GiB budget at `rates` and with a 1 GiB
    budget (admission binds) at `rates_small`."""
    log(f"served: preparing {nreq} requests (input hashes, oracle sample)")
    st = ServedTrace(binding, torch, np, inputs, pools_dev, pools_host, nreq)
    res = {"requests": nreq, "keys_per_sweep_point": st.total_keys, "pool_keys": st.pool_keys,
           "sample_requests": int(st.sample.size), "alone_min_keys": alone_min_keys,
           "checks": "every output: no descent and SplitMix64 sum/xor equal to its input's (on the device); "
                     "a seeded 1% sample of requests: keys and splitters bit-exact against the oracle"}
    cap = run_plain(st, None, closed_loop=True)
    plain_cap = cap["req_s"]
    res["plain_fifo_closed_loop"] = cap
    log(f"served: plain capacity {cap}")
    res["points"] = []
    with binding.Server(hbm_budget_bytes=64 << 30, num_streams=4, max_batch=256, alone_min_keys=alone_min_keys) as srv:
        for frac in rates:
            arr = st.arrivals(frac * plain_cap)
            served = run_served(st, srv, arr)
            plain = run_plain(st, arr)
            res["points"].append({"offered_frac_of_plain_capacity": frac, "offered_req_s": round(frac * plain_cap, 1),
                                  "served": served, "plain_fifo": plain})
            log(f"served frac={frac}: {res['points'][-1]}")
    res["budget_1GiB"] = []
    with binding.Server(hbm_budget_bytes=1 << 30, num_streams=4, max_batch=256, alone_min_keys=alone_min_keys) as srv:
        for frac in rates_small:
            served = run_served(st, srv, st.arrivals(frac * plain_cap))
            res["budget_1GiB"].append({"offered_frac_of_plain_capacity": frac, "served": served})
            log(f"served 1 GiB budget frac={frac}: {served}")
    bad = sum(p["served"]["outputs_bad"] + p["plain_fifo"]["outputs_bad"] + p["served"]["sample_keys_bad"]
              + p["served"]["sample_splitters_bad"] for p in res["points"])
    bad += sum(p["served"]["outputs_bad"] + p["served"]["sample_keys_bad"] + p["served"]["sample_splitters_bad"]
               for p in res["budget_1GiB"])
    res["all_outputs_ok"] = bad == 0
    del st
    return res


# ------------------------------------------------------------------------------------------------
def host_description() -> dict:
    """nproc, the threads this process may use, and the CPU model of the host."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": os.cpu_count(), "threads_allowed": allowed, "cpu_model": model}


def cpu_baseline(keys, max_s: float = 10.0, max_reps: int = 8) -> dict:
    """The CPU oracle on the benchmark's 2^26 keys: the single-thread LSD sort and the same passes
    split over every thread the process may use (at most 16, the host share of one GPU); each
    timed over up to `max_reps` full sorts or `max_s` seconds."""
    import oracle
    host = host_description()
    threads = max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or host["threads_allowed"] or 1,
                         host["threads_allowed"] or 1))

    def rate(fn):
        fn(keys[:4096])
        reps, t0 = 0, time.perf_counter()
        while True:
            fn(keys)
            reps += 1
            el = time.perf_counter() - t0
            if el > max_s or reps >= max_reps:
                return reps, keys.size * reps / el / 1e9

    reps1, one = rate(oracle.sort_u32)
    repsm, many = rate(lambda k: oracle.sort_u32_mt(k, threads))
    return {"value": round(many, 5), "unit": "Gkeys/s", "cores": threads, "kind": "oracle",
            "sample": f"{repsm} full sorts of the benchmark's 2^26 uniform keys (seed 1), every pass split over "
                      f"{threads} threads; single thread: {reps1} sorts",
            "single_core": {"value": round(one, 5), "cores": 1}, "host": host}


# ------------------------------------------------------------------------------------------------
def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip every extra leg")
    ap.add_argument("--no-dists", action="store_true", help="skip distributions (b)-(e) and the 2^27 sets")
    ap.add_argument("--no-segmented", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=100_000)
    ap.add_argument("--served-rates", default="0.25,0.5,0.75,0.9,1.0,1.25,2.0",
                    help="offered rates (fractions of the plain form's capacity), 64 GiB server budget")
    ap.add_argument("--served-rates-1g", default="0.5,1.0,1.25,2.0",
                    help="offered rates with a 1 GiB server budget (admission binds)")
    ap.add_argument("--alone-min-keys", type=int, default=1 << 16,
                    help="served form: requests with at least this many keys run the device-wide sort alone")
    ap.add_argument("--profile-leg", choices=["segmented", "segmented-long", "msd", "latency", "merge"], default=None,
                    help="run only that leg (for rocprofv3) and print its result")
    ap.add_argument("--msd-dists", default="a,e",
                    help="distributions of the msd profile leg (three sorts of 2^26 keys each)")
    ap.add_argument("--phase-trace", action="store_true",
                    help="print per-phase tile durations of k_pass at 2^26 (ap_debug_pass trace mode) as markdown")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the sort runs on one GPU only (asked for --gpus {args.gpus}); it is sized for one "
              "device's HBM and has no multi-GPU path",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_cs_0004013_amd import binding, inputs

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.copy_calib:
        a = torch.empty(N_MAIN, dtype=torch.int32, device="cuda").fill_(7)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": 4 * N_MAIN, "copy_calib_bytes_written": 4 * N_MAIN,
                          "launches": 5}), flush=True)
        return 0
    binding.lib()
    if args.phase_trace:
        print(phase_trace(binding, torch, np, inputs), flush=True)
        return 0
    if args.profile_leg == "segmented":
        print(json.dumps(leg_segmented(binding, torch, np, inputs, steps=3, baseline=False)), flush=True)
        return 0
    if args.profile_leg == "segmented-long":
        spl = torch.empty(63, dtype=torch.int32, device="cuda")
        print(json.dumps(leg_segmented_long(binding, torch, np, inputs, spl, steps=3)), flush=True)
        return 0
    if args.profile_leg == "msd":
        # the bucketing variant alone (three sorts of 2^26 keys per distribution), for its counters;
        # each output checked on the device (no descent, same multiset hash as the input)
        spl = torch.empty(63, dtype=torch.int32, device="cuda")
        res = {}
        for dist in args.msd_dists.split(","):
            t_in = torch.from_numpy(inputs.keyset(dist, N_MAIN, seed=1).keys.view(np.int32)).to("cuda")
            out = torch.empty_like(t_in)
            for _ in range(3):
                binding.ap_sort_u32_msd(t_in, out, 64, spl)
            acc = torch.zeros((2, 3), dtype=torch.int64, device="cuda")
            binding.ap_check_u32(t_in, acc[0])
            binding.ap_check_u32(out, acc[1])
            a = acc.cpu().numpy()
            res[dist] = bool(a[1, 0] == 0 and a[0, 1] == a[1, 1] and a[0, 2] == a[1, 2])
        print(json.dumps({"msd_sorted": res}), flush=True)
        return 0
    if args.profile_leg == "latency":
        print(json.dumps(leg_latency(binding, torch, np, inputs)), flush=True)
        return 0
    if args.profile_leg == "merge":
        t_keys = torch.from_numpy(inputs.keyset("a", N_MAIN, seed=1).keys.view(np.int32)).to("cuda")
        print(json.dumps(leg_merge(binding, torch, np, inputs, t_keys, steps=3)), flush=True)
        return 0

    def upload(keys):
        return torch.from_numpy(keys.view(np.int32)).to("cuda")

    log("generating 2^26 uniform keys (seed 1)")
    ks = inputs.keyset("a", N_MAIN, seed=1)
    t_in = upload(ks.keys)
    t_out = torch.empty_like(t_in)
    spl = torch.empty(63, dtype=torch.int32, device="cuda")

    log(f"timing {args.steps} steps after {args.warmup} warm-up")
    dt, _ = time_sorts(binding, torch, t_in, t_out, spl, args.steps, args.warmup, False)
    ms_per_step = dt * 1e3 / args.steps
    value = N_MAIN * args.steps / dt / 1e9
    # per-kernel durations: the same sorts again with HIP events around every launch
    _, prof = time_sorts(binding, torch, t_in, t_out, spl, args.steps, 1, True)
    ms, launches = prof
    pass_avg_s = pass_stats(binding, prof)
    alg_bytes = 8 * N_MAIN                      # one pass reads and writes every key once
    achieved = alg_bytes / pass_avg_s / 1e9
    profile = read_profile()
    per_kernel_us = {
        "k_hist_plan": ms[binding.AP_KIND_HIST] / max(launches[binding.AP_KIND_HIST], 1) * 1e3,
        "k_pass": pass_avg_s * 1e6,
        "k_finalize": ms[binding.AP_KIND_FINAL] / max(launches[binding.AP_KIND_FINAL], 1) * 1e3,
    }

    extra = {}
    # measured ceiling of a plain device copy of the same bytes (context for the 8 TB/s peak)
    cbuf = torch.empty_like(t_in)
    cs = torch.cuda.current_stream()
    for _ in range(3):
        cbuf.copy_(t_in)
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record(cs)
    for _ in range(10):
        cbuf.copy_(t_in)
    ce1.record(cs)
    torch.cuda.synchronize()
    copy_gbs = 10 * 8 * N_MAIN / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
    del cbuf
    pools = {"a": t_in}
    pools_host = {"a": ks.keys}
    if not args.no_extra and not args.no_dists:
        for seed, dist in zip(range(2, 6), "bcde"):
            log(f"distribution ({dist}) seed {seed}")
            hk = inputs.keyset(dist, N_MAIN, seed=seed).keys
            k2 = upload(hk)
            o2 = torch.empty_like(k2)
            d2, _ = time_sorts(binding, torch, k2, o2, spl, 10, 3, False)
            extra[f"dist_{dist}_gkeys_s"] = round(N_MAIN * 10 / d2 / 1e9, 3)
            pools[dist], pools_host[dist] = k2, hk
            del o2
        log("adversarial 2^27")
        k3 = upload(inputs.adversarial(1 << 27, seed=0).keys)
        o3 = torch.empty_like(k3)
        d3, _ = time_sorts(binding, torch, k3, o3, spl, 5, 2, False)
        extra["adversarial_2p27_gkeys_s"] = round((1 << 27) * 5 / d3 / 1e9, 3)
        del k3, o3
        log("uniform 2^27: per-pass roofline")
        extra["uniform_2p27"] = leg_pass_2p27(binding, torch, np, inputs, spl)
        log("bucketing variant (MSD) vs LSD")
        extra["msd_vs_lsd_2p26"] = leg_msd(binding, torch, np, pools, spl)
    if not args.no_extra:
        log("merge 2 x 2^25")
        extra["merge_2x2p25"] = leg_merge(binding, torch, np, inputs, t_in)
        log("pairs 2^26")
        extra["pairs_2p26"] = leg_pairs(binding, torch, np, inputs, t_in)
        log("latency 2^20")
        extra["latency_2p20"] = leg_latency(binding, torch, np, inputs)
    if not args.no_extra and not args.no_segmented:
        log("segmented 4096-segment batch")
        extra["segmented_4096"] = leg_segmented(binding, torch, np, inputs, steps=5)
        log("segmented: long segments")
        extra["segmented_long"] = leg_segmented_long(binding, torch, np, inputs, spl)
    if not args.no_extra and not args.no_served:
        for seed, dist in zip(range(2, 6), "bcde"):
            if dist not in pools:
                pools_host[dist] = inputs.keyset(dist, N_MAIN, seed=seed).keys
                pools[dist] = upload(pools_host[dist])
        log("served form")
        rates = [float(x) for x in args.served_rates.split(",") if x]
        rates_small = [float(x) for x in args.served_rates_1g.split(",") if x]
        extra["served"] = leg_served(binding, torch, np, inputs, pools, pools_host, args.served_requests, rates,
                                     rates_small, args.alone_min_keys)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline(ks.keys)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "sort 2^26 u32 keys uniform in [0,2^31-1] (dist a, seed 1) into 64 cells "
                               "+ 63 splitters, keys resident in HBM",
                   "n": N_MAIN, "P": 64, "digit_bits": 8, "passes": 4},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profile["traffic"] if profile else None,
                     "kernel": "k_pass", "alg_bytes_per_launch": alg_bytes, "timer": "hip_events",
                     "rocprof_mean_us": profile["mean_us"] if profile else None,
                     "frac_rocprof": round(alg_bytes / profile["mean_us"] / 1e3 / HBM_PEAK_GBS, 4) if profile else None,
                     "copy_ceiling_gbs": round(copy_gbs, 1), "frac_of_copy_ceiling": round(achieved / copy_gbs, 4)},
        "cpu_baseline": cpu,
        "per_kernel_us": {k: round(v, 2) for k, v in per_kernel_us.items()},
        **extra,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
