"""Autotuner of the segmented sort: picks the kernel configuration (digit width, waves per
workgroup, keys per lane) of each length group by measurement.

The length groups are fixed ranges of length classes ceil(log2(segment length)), one per tile
size: more than 8K keys (16K-key tiles, longer segments by digit sweeps), (4K, 8K], (2K, 4K] and
up to 2K.  Every group is one more concurrent persistent kernel: classes that run the same
configuration are better served by one group (a fifth group splitting off the segments above 16K
measured 1.5-2% slower with the same configurations).  The tuning batch has the workload's shape: 4096 segments with lengths
log-uniform in [64, 2^18] and distributions (a)-(e) by segment seed; three such batches are
drawn with seeds of their own (not the benchmark's), because which configuration wins depends on
the particular lengths (the longest segments set the critical path).  The groups are tuned by
coordinate descent: for one group at a time, every compiled-in configuration is tried with the
other groups' choices fixed, scored by the sum over the batches of the median of `reps` runs
(input restored before each run, HIP events on the sort's stream); the lowest score is kept, and
the sweep over the groups is repeated `rounds` times.  (Tuning each group on
a batch of its own lengths alone picks differently: it misses how many segments of each length
the workload has, and with it how much parallelism each group's kernel gets.)  The result is
written as lines "group cls_lo cls_hi cfg" that the library reads with ap_load_tuning.

Usage (on the GPU):  python -m paper_cs_0004013_amd.autotune [--out FILE] [--reps R] [--rounds N]
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tune_gfx950.txt")
GROUPS = [(14, 31), (13, 13), (12, 12), (1, 11)]   # > 8K, (4K, 8K], (2K, 4K], <= 2K keys
START = [10, 0, 5, 3]                               # configurations the descent starts from (the built-in table)
TUNE_SEEDS = (7919, 104729, 1299709)


def _batch(seed: int):
    from paper_cs_0004013_amd import inputs
    L = inputs.segment_lengths(4096, seed=seed)
    keys, off, _ = inputs.segment_keys(L)
    return keys, off


def tune(reps: int = 5, rounds: int = 2, out: str | None = DEFAULT_TABLE, verbose: bool = True):
    import torch

    from paper_cs_0004013_amd import binding

    binding.lib()
    saved = binding.segmented_groups()
    ncfg = binding.ap_segmented_num_configs()
    stream = torch.cuda.Stream()
    batches = [_batch(sd) for sd in TUNE_SEEDS]
    nkeys = sum(int(k.size) for k, _ in batches)
    choice = list(START)
    try:
        with torch.cuda.stream(stream):
            dev = [(torch.from_numpy(k.view(np.int32)).to("cuda"), torch.from_numpy(o.view(np.int32)).to("cuda"))
                   for k, o in batches]
            t_work = torch.empty(max(int(k.size) for k, _ in batches), dtype=torch.int32, device="cuda")

            def measure() -> float:
                binding.set_segmented_groups([(lo, hi, c) for (lo, hi), c in zip(GROUPS, choice)])
                total = 0.0
                for t_src, t_off in dev:
                    work = t_work[:t_src.numel()]
                    times = []
                    for r in range(reps + 1):
                        work.copy_(t_src)
                        a = torch.cuda.Event(enable_timing=True)
                        b = torch.cuda.Event(enable_timing=True)
                        a.record(stream)
                        binding.ap_sort_u32_segmented(work, t_off, stream=stream)
                        b.record(stream)
                        stream.synchronize()
                        if r:
                            times.append(a.elapsed_time(b))
                    total += float(np.median(times))
                return total

            best = measure()
            if verbose:
                print(f"[tune] {len(dev)} batches of 4096 segments, {nkeys} keys; start {choice}: {best:.3f} ms",
                      flush=True)
            for rnd in range(rounds):
                for g in range(len(GROUPS)):
                    for cfg in range(ncfg):
                        if cfg == choice[g]:
                            continue
                        prev = choice[g]
                        choice[g] = cfg
                        ms = measure()
                        if verbose:
                            bits, waves, ipt = binding.ap_segmented_config_info(cfg)
                            print(f"[tune] round {rnd} group {g} classes {GROUPS[g][0]}..{GROUPS[g][1]} cfg {cfg} "
                                  f"(bits {bits}, waves {waves}, ipt {ipt}): {ms:.3f} ms", flush=True)
                        if ms < best * 0.995:
                            best = ms
                        else:
                            choice[g] = prev
                if verbose:
                    print(f"[tune] after round {rnd}: {choice} {best:.3f} ms "
                          f"({nkeys / best / 1e6:.1f} Gkeys/s)", flush=True)
    finally:
        binding.set_segmented_groups(saved)
    chosen = [(lo, hi, c) for (lo, hi), c in zip(GROUPS, choice)]
    if out:
        with open(out, "w") as f:
            f.write("# segmented-sort length groups: group cls_lo cls_hi cfg  (ceil(log2 length) classes)\n")
            f.write("# written by paper_cs_0004013_amd.autotune (coordinate descent on three 4096-segment batches)\n")
            for g, (lo, hi, cfg) in enumerate(chosen):
                f.write(f"{g} {lo} {hi} {cfg}\n")
        if verbose:
            print(f"[tune] wrote {out}", flush=True)
    return chosen


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--rounds", type=int, default=2)
    args = ap.parse_args()
    tune(args.reps, args.rounds, args.out)
    return 0


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    sys.exit(main())
