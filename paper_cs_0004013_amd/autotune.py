"""Autotuner of the segmented sort: picks the kernel configuration (digit width, waves per
workgroup, keys per lane) of each length group by measurement.

For each length group (a range of floor(log2(segment length)) classes) a synthetic batch whose
lengths all fall in that group is built (log-uniform lengths, distributions (a)-(e) by segment
seed, about 2^25 keys in total).  With the group table reduced to that one group, every compiled-in
configuration sorts the batch (input restored before each run; HIP events on the sort's stream),
and the configuration with the lowest median time is kept.  The result is written as a table of
lines "group cls_lo cls_hi cfg" that the library reads with ap_load_tuning.

Usage (on the GPU):  python -m paper_cs_0004013_amd.autotune [--out FILE] [--reps R]
"""
from __future__ import annotations

import argparse
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tune_gfx950.txt")
GROUPS = [(13, 18), (11, 12), (1, 10)]   # >= 8192, 2048..8191, 2..2047 keys (segments up to 2^18 tuned)
TARGET_KEYS = 1 << 25


def _batch_for(cls_lo: int, cls_hi: int, seed: int):
    from paper_cs_0004013_amd import inputs
    lo, hi = 1 << cls_lo, (1 << (cls_hi + 1)) - 1
    mean = (hi - lo) / max(math.log(hi / lo), 1e-9)
    nseg = int(min(max(TARGET_KEYS / mean, 64), 65536))
    L = inputs.segment_lengths(nseg, seed=seed, lo=max(lo, 2), hi=hi)
    keys, off, _ = inputs.segment_keys(L)
    return keys, off


def tune(reps: int = 5, out: str | None = DEFAULT_TABLE, verbose: bool = True) -> list[tuple[int, int, int]]:
    import torch

    from paper_cs_0004013_amd import binding

    binding.lib()
    saved = binding.segmented_groups()
    ncfg = binding.ap_segmented_num_configs()
    stream = torch.cuda.Stream()
    chosen = []
    try:
        for gi, (cls_lo, cls_hi) in enumerate(GROUPS):
            keys, off = _batch_for(cls_lo, cls_hi, seed=1000 + gi)
            with torch.cuda.stream(stream):
                t_src = torch.from_numpy(keys.view(np.int32)).to("cuda")
                t_work = torch.empty_like(t_src)
                t_off = torch.from_numpy(off.view(np.int32)).to("cuda")
                best = None
                for cfg in range(ncfg):
                    binding.set_segmented_groups([(cls_lo, cls_hi, cfg)] + [(1, 0, 0)] * (binding.SEG_GROUPS - 1))
                    times = []
                    for r in range(reps + 1):
                        t_work.copy_(t_src)
                        a = torch.cuda.Event(enable_timing=True)
                        b = torch.cuda.Event(enable_timing=True)
                        a.record(stream)
                        binding.ap_sort_u32_segmented(t_work, t_off, stream=stream)
                        b.record(stream)
                        stream.synchronize()
                        if r:
                            times.append(a.elapsed_time(b))
                    ms = float(np.median(times))
                    bits, waves, ipt = binding.ap_segmented_config_info(cfg)
                    if verbose:
                        print(f"[tune] group {gi} classes {cls_lo}..{cls_hi} ({keys.size} keys, {off.size - 1} segs) "
                              f"cfg {cfg} (bits {bits}, waves {waves}, ipt {ipt}): {ms:.3f} ms "
                              f"{keys.size / ms / 1e6:.1f} Gkeys/s", flush=True)
                    if best is None or ms < best[0]:
                        best = (ms, cfg)
            chosen.append((cls_lo, cls_hi, best[1]))
    finally:
        binding.set_segmented_groups(saved)
    # the top group also covers lengths beyond the tuned range
    chosen[0] = (chosen[0][0], 31, chosen[0][2])
    if out:
        with open(out, "w") as f:
            f.write("# segmented-sort length groups: group cls_lo cls_hi cfg  (floor(log2 length) classes)\n")
            f.write("# written by paper_cs_0004013_amd.autotune on the GPU it ran on\n")
            for g, (lo, hi, cfg) in enumerate(chosen):
                f.write(f"{g} {lo} {hi} {cfg}\n")
        if verbose:
            print(f"[tune] wrote {out}", flush=True)
    return chosen


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    tune(args.reps, args.out)
    return 0


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    sys.exit(main())
