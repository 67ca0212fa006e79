#!/usr/bin/env python3
"""Benchmark of the radix sort on one MI355X.

A step is one full sort (bucket counts + plan, every digit pass, splitters) of 2^26 uint32 keys,
i.i.d. uniform in [0, 2^31-1] (distribution (a), seed 1), already resident in HBM, into P = 64 cells.
`value` is keys sorted per second over the K timed steps (Gkeys/s).  The roofline object describes
the digit-pass kernel (k_pass), timed with HIP events recorded around each launch on the sort's
stream during the timed steps.  The other distributions (b)-(e) at 2^26 and the adversarial 2^27
set are reported as extra fields.  The CPU baseline is the oracle (plain single-threaded C LSD
radix sort) on the same 2^26-key array.

Prints ONE JSON line.
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
KERNEL_SRC = os.path.join(ROOT, "paper_cs_0004013_amd", "csrc", "apsort_kernels.h")
COUNTERS = os.path.join(ROOT, "profiles", "k_pass_counters_uniform_2p26.md")


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the other distributions")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the sort "
              "is sized for one device's HBM and has no multi-GPU path", file=sys.stderr)
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

    def upload(keys):
        return torch.from_numpy(keys.view(np.int32)).to("cuda")

    log("generating 2^26 uniform keys (seed 1)")
    ks = inputs.keyset("a", N_MAIN, seed=1)
    t_in = upload(ks.keys)
    t_out = torch.empty_like(t_in)
    spl = torch.empty(63, dtype=torch.int32, device="cuda")

    log(f"timing {args.steps} steps after {args.warmup} warm-up")
    dt, (ms, launches) = time_sorts(binding, torch, t_in, t_out, spl, args.steps, args.warmup, True)
    ms_per_step = dt * 1e3 / args.steps
    value = N_MAIN * args.steps / dt / 1e9

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
    if not args.no_extra:
        for seed, dist in zip(range(2, 6), "bcde"):
            log(f"distribution ({dist}) seed {seed}")
            k2 = upload(inputs.keyset(dist, N_MAIN, seed=seed).keys)
            o2 = torch.empty_like(k2)
            d2, _ = time_sorts(binding, torch, k2, o2, spl, 10, 3, False)
            extra[f"dist_{dist}_gkeys_s"] = round(N_MAIN * 10 / d2 / 1e9, 3)
            del k2, o2
        log("adversarial 2^27")
        k3 = upload(inputs.adversarial(1 << 27, seed=0).keys)
        o3 = torch.empty_like(k3)
        d3, (ms3, l3) = time_sorts(binding, torch, k3, o3, spl, 5, 2, True)
        extra["adversarial_2p27_gkeys_s"] = round((1 << 27) * 5 / d3 / 1e9, 3)
        del k3, o3

    cpu = None
    if not args.no_cpu:
        import oracle
        log("CPU oracle baseline")
        oracle.sort_u32(ks.keys[:1024])
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.sort_u32(ks.keys)
            reps += 1
            el = time.perf_counter() - t0
            if el > 10.0 or reps >= 8:
                break
        cpu = {"value": round(N_MAIN * reps / el / 1e9, 5), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full sorts of the same 2^26 uniform keys (seed 1), single thread"}

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
                     "kernel": "k_pass", "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "per_kernel_us": {k: round(v, 2) for k, v in per_kernel_us.items()},
        **extra,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
