#!/usr/bin/env python3
"""Benchmark of the radix sort on one MI355X.  Prints ONE JSON line.

Main metric: a step is one full sort (bucket counts + plan, every digit pass, splitters) of 2^26
uint32 keys, i.i.d. uniform in [0, 2^31-1] (distribution (a), seed 1), already resident in HBM,
into P = 64 cells; `value` is keys sorted per second over the K timed steps (Gkeys/s).

`roofline` describes the digit-pass kernel k_pass: algorithmic bytes per launch (8 B per key) over
the mean launch duration, timed with HIP events recorded around each launch on the sort's stream
during the timed steps.  `traffic` comes from the committed rocprofv3 counter summary when it was
taken on the current kernel source.

Extra fields (each can be skipped): the other distributions (b)-(e) at 2^26 and the adversarial
2^27 set; the 4096-segment batch (lengths log-uniform in [64, 2^18]) sorted by the batched
segmented form vs a loop of plain per-array launches; the served form (Poisson arrivals of
log-uniform [2^10, 2^24] requests at several rates) vs one plain launch per request, FIFO on one
stream; p50/p99 latency of a 2^20-key sort.  The CPU baseline is the oracle (plain C LSD radix
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
# the pass kernel and the device helpers it inlines (rank, look-back words)
KERNEL_SRCS = [os.path.join(ROOT, "paper_cs_0004013_amd", "csrc", f) for f in ("apsort_kernels.h", "apsort_device.h")]
COUNTERS = os.path.join(ROOT, "profiles", "k_pass_counters_uniform_2p26.md")


def kernel_sha() -> str:
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SRCS)).hexdigest()[:16]


def read_traffic():
    """HBM bytes per k_pass launch from the committed rocprofv3 counter summary, or None when the
    summary is missing or was taken on a different kernel source."""
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
        return float(vals["hbm_bytes_per_launch"])
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


def pct(v, p):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), p)) if len(v) else None


# ------------------------------------------------------------------------------------------------
def leg_latency(binding, torch, np, inputs):
    """2^20 uniform keys (seed 0), 64 cells: per-sort latency over 50 timed sorts."""
    keys = inputs.keyset("a", 1 << 20, seed=0).keys
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
    return {"n": 1 << 20, "p50_ms": round(pct(ms, 50), 4), "p99_ms": round(pct(ms, 99), 4),
            "gkeys_s_p50": round((1 << 20) / pct(ms, 50) / 1e6, 2)}


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
    ms, cnt = binding.ap_profile_read()
    npass = sum(cnt[binding.AP_KIND_PASS + d] for d in range(4))
    pass_us = sum(ms[binding.AP_KIND_PASS + d] for d in range(4)) / max(npass, 1) * 1e3
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


def leg_segmented(binding, torch, np, inputs, steps: int, baseline: bool = True):
    """4096 segments, lengths log-uniform in [64, 2^18] (seed 0); segment s uses seed s."""
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
        got = t_work.cpu().numpy().view(np.uint32)
        # cheap full check: nondecreasing inside every segment, multiset kept per segment boundary
        d = np.diff(got.astype(np.int64))
        inside = np.ones(n - 1, dtype=bool)
        inside[off[1:-1].astype(np.int64) - 1] = False
        ok = bool(np.all(d[inside] >= 0)) and int(got.astype(np.uint64).sum()) == int(keys.astype(np.uint64).sum())
        res["segments"] = 4096
        res["keys"] = n
        res["batched_ms_p50"] = round(pct(ms, 50), 4)
        res["batched_gkeys_s"] = round(n / pct(ms, 50) / 1e6, 3)
        res["batched_ok"] = ok
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


def leg_served(binding, torch, np, inputs, pools_dev, nreq: int, rates, alone_min_keys: int = 1 << 16):
    """Poisson trace of nreq requests (sizes log-uniform [2^10, 2^24], distribution and pool
    window by request seed) served by the request server at several offered rates, and the same
    trace as one plain launch per request, FIFO on one stream."""
    pool_keys = int(next(iter(pools_dev.values())).numel())
    ring = 128                                 # output buffers reused round-robin
    outs = [torch.empty(1 << 24, dtype=torch.int32, device="cuda") for _ in range(ring)]
    spls = [torch.empty(63, dtype=torch.int32, device="cuda") for _ in range(ring)]
    lib = binding.lib()
    res = {"requests": nreq, "pool_keys": pool_keys}

    # -- baseline: plain launches back to back (closed loop) gives the capacity, then its latency
    base_trace = inputs.request_trace(nreq, rate_per_s=1.0, pool_keys=pool_keys, seed=0)
    total_keys = sum(r.n for r in base_trace)
    s = torch.cuda.Stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nreq)]
    start = torch.cuda.Event(enable_timing=True)
    start.record(s)
    t0 = time.perf_counter()
    for i, r in enumerate(base_trace):
        src = pools_dev[r.dist][r.pool_offset:r.pool_offset + r.n]
        st = lib.ap_sort_u32(src.data_ptr(), outs[i % ring].data_ptr(), r.n, 64, spls[i % ring].data_ptr(),
                             s.cuda_stream)
        if st:
            raise RuntimeError(binding.last_error())
        evs[i].record(s)
    s.synchronize()
    t_plain = time.perf_counter() - t0
    plain_cap = nreq / t_plain
    res["plain_fifo_closed_loop"] = {"req_s": round(plain_cap, 1), "gkeys_s": round(total_keys / t_plain / 1e9, 3)}

    # -- served, open loop at rates relative to the plain capacity; plain FIFO at the same rates
    def run_served(srv, tr):
        st0 = srv.stats(reset_latencies=True)
        tickets = [0] * nreq
        t0 = time.perf_counter()
        for i, r in enumerate(tr):
            while time.perf_counter() - t0 < r.arrival_s:
                pass
            if i >= ring:
                st = srv.wait(tickets[i - ring])  # output buffer reuse
                if st:
                    raise RuntimeError(f"request failed: {st}")
            src = pools_dev[r.dist][r.pool_offset:r.pool_offset + r.n]
            tickets[i] = srv.submit_ptr(src.data_ptr(), outs[i % ring].data_ptr(), r.n, 64,
                                        spls[i % ring].data_ptr())
        for i in range(max(0, nreq - ring), nreq):
            st = srv.wait(tickets[i])
            if st:
                raise RuntimeError(f"request failed: {st}")
        wall = time.perf_counter() - t0
        stt = srv.stats(reset_latencies=True)
        # the last `ring` outputs are still in place: compare them with torch's sort of the input
        # window (keys < 2^31, so int32 order is the unsigned order), after the timed region
        checked, bad = 0, 0
        for i in range(max(0, nreq - ring), nreq):
            r = tr[i]
            src = pools_dev[r.dist][r.pool_offset:r.pool_offset + r.n]
            want = torch.sort(src)[0]
            bad += int(not torch.equal(outs[i % ring][:r.n], want))
            checked += 1
        return {"gkeys_s": round(sum(r.n for r in tr) / wall / 1e9, 3), "p50_ms": round(stt["p50_us"] / 1e3, 4),
                "p99_ms": round(stt["p99_us"] / 1e3, 4), "batches": stt["batches"] - st0["batches"],
                "alone": stt["alone"] - st0["alone"], "outputs_checked": checked, "outputs_bad": bad}

    res["points"] = []
    res["alone_min_keys"] = alone_min_keys
    with binding.Server(hbm_budget_bytes=64 << 30, num_streams=4, max_batch=256, alone_min_keys=alone_min_keys) as srv:
        for frac in rates:
            lam = frac * plain_cap
            tr = inputs.request_trace(nreq, rate_per_s=lam, pool_keys=pool_keys, seed=0)
            served = run_served(srv, tr)
            # plain FIFO at the same offered rate: latency = completion event - arrival
            start = torch.cuda.Event(enable_timing=True)
            t1 = time.perf_counter()
            start.record(s)
            for i, r in enumerate(tr):
                while time.perf_counter() - t1 < r.arrival_s:
                    pass
                src = pools_dev[r.dist][r.pool_offset:r.pool_offset + r.n]
                lib.ap_sort_u32(src.data_ptr(), outs[i % ring].data_ptr(), r.n, 64, spls[i % ring].data_ptr(),
                                s.cuda_stream)
                evs[i].record(s)
            s.synchronize()
            wall_p = time.perf_counter() - t1
            lat_p = [start.elapsed_time(evs[i]) - tr[i].arrival_s * 1e3 for i in range(nreq)]
            res["points"].append({
                "offered_frac_of_plain_capacity": frac,
                "offered_req_s": round(lam, 1),
                "served": served,
                "plain_fifo": {"gkeys_s": round(sum(r.n for r in tr) / wall_p / 1e9, 3),
                               "p50_ms": round(pct(lat_p, 50), 4), "p99_ms": round(pct(lat_p, 99), 4)},
            })
            log(f"served frac={frac}: {res['points'][-1]}")
    # a 1 GiB budget (256 MiB of scratch per slot) so that admission binds, at 1.25x
    with binding.Server(hbm_budget_bytes=1 << 30, num_streams=4, max_batch=256, alone_min_keys=alone_min_keys) as srv:
        tr = inputs.request_trace(nreq, rate_per_s=1.25 * plain_cap, pool_keys=pool_keys, seed=0)
        res["budget_1GiB_at_1.25"] = run_served(srv, tr)
        log(f"served 1 GiB budget: {res['budget_1GiB_at_1.25']}")
    return res


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
    ap.add_argument("--no-dists", action="store_true", help="skip distributions (b)-(e) and the 2^27 set")
    ap.add_argument("--no-segmented", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=20000)
    ap.add_argument("--served-rates", default="0.5,0.9,1.25,2.0")
    ap.add_argument("--alone-min-keys", type=int, default=1 << 16,
                    help="served form: requests with at least this many keys run the device-wide sort alone")
    ap.add_argument("--profile-leg", choices=["segmented", "latency", "merge"], default=None,
                    help="run only that leg (for rocprofv3) and print its result")
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
    if args.profile_leg == "segmented":
        print(json.dumps(leg_segmented(binding, torch, np, inputs, steps=3, baseline=False)), flush=True)
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
    _, (ms, launches) = time_sorts(binding, torch, t_in, t_out, spl, args.steps, 1, True)

    pass_ms = sum(ms[binding.AP_KIND_PASS + d] for d in range(4))
    pass_launches = sum(launches[binding.AP_KIND_PASS + d] for d in range(4))
    pass_avg_s = pass_ms / pass_launches / 1e3
    alg_bytes = 8 * N_MAIN                      # one pass reads and writes every key once
    achieved = alg_bytes / pass_avg_s / 1e9
    traffic = read_traffic()
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
    if not args.no_extra and not args.no_dists:
        for seed, dist in zip(range(2, 6), "bcde"):
            log(f"distribution ({dist}) seed {seed}")
            k2 = upload(inputs.keyset(dist, N_MAIN, seed=seed).keys)
            o2 = torch.empty_like(k2)
            d2, _ = time_sorts(binding, torch, k2, o2, spl, 10, 3, False)
            extra[f"dist_{dist}_gkeys_s"] = round(N_MAIN * 10 / d2 / 1e9, 3)
            pools[dist] = k2
            del o2
        log("adversarial 2^27")
        k3 = upload(inputs.adversarial(1 << 27, seed=0).keys)
        o3 = torch.empty_like(k3)
        d3, _ = time_sorts(binding, torch, k3, o3, spl, 5, 2, False)
        extra["adversarial_2p27_gkeys_s"] = round((1 << 27) * 5 / d3 / 1e9, 3)
        del k3, o3
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
    if not args.no_extra and not args.no_served:
        for seed, dist in zip(range(2, 6), "bcde"):
            if dist not in pools:
                pools[dist] = upload(inputs.keyset(dist, N_MAIN, seed=seed).keys)
        log("served form")
        rates = [float(x) for x in args.served_rates.split(",") if x]
        extra["served"] = leg_served(binding, torch, np, inputs, pools, args.served_requests, rates,
                                     args.alone_min_keys)

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
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_pass", "alg_bytes_per_launch": alg_bytes,
                     "copy_ceiling_gbs": round(copy_gbs, 1), "frac_of_copy_ceiling": round(achieved / copy_gbs, 4)},
        "cpu_baseline": cpu,
        "per_kernel_us": {k: round(v, 2) for k, v in per_kernel_us.items()},
        **extra,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
