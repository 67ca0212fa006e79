"""Turn rocprofv3 result databases into the short text summaries kept under profiles/.

Usage (after the rocprofv3 runs named in the summary header):
  python -m paper_cs_0004013_amd.profile_summary --trace DIR --fetch DIR --write DIR \
      --fetch-copy DIR --write-copy DIR --kernel k_pass --out profiles/NAME.md --cmd "..."

Each DIR holds one rocprofv3 run (its *_results.db).  The summary lists the mean duration of every
kernel of the trace run, and for the named kernel the FETCH_SIZE and WRITE_SIZE per dispatch,
each scaled by the factor that makes the same counter read the known size of a plain 256 MiB
device copy (the copy-calibration runs), giving HBM bytes per launch.  It records a hash of the
kernel's sources (--source, comma-separated; default apsort_kernels.h and the device helpers of
apsort_device.h) so that bench.py can tell whether the counters still describe the current kernel.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import os
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = ",".join(os.path.join(HERE, "csrc", f)
                      for f in ("apsort_kernels.h", "apsort_pass_core.h", "apsort_device.h"))
COPY_BYTES = 4 * (1 << 26)


def _db(d: str) -> sqlite3.Connection:
    files = glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no rocprofv3 results database under {d}")
    return sqlite3.connect(files[0])


def kernel_times(d: str) -> list[tuple[str, int, float]]:
    con = _db(d)
    rows = con.execute("select name, total_calls, average from top_kernels").fetchall()
    return [(r[0], int(r[1]), float(r[2])) for r in rows]  # average is in microseconds


def _match(name: str, kernel_substr: str, exclude: tuple[str, ...] = ()) -> bool:
    return kernel_substr in name and not any(x in name for x in exclude)


def counter_per_dispatch(d: str, counter: str, kernel_substr: str,
                         exclude: tuple[str, ...] = ()) -> tuple[float, int]:
    """Mean of the counter over the dispatches of kernels whose name contains kernel_substr (and
    none of the `exclude` substrings).  rocprofv3 reports the value per dispatch (summed over the
    device's instances)."""
    con = _db(d)
    rows = con.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                       "where counter_name = ? group by dispatch_id", (counter,)).fetchall()
    vals = [float(v) for name, _, v in rows if _match(name, kernel_substr, exclude)]
    if not vals:
        raise ValueError(f"no {counter} samples for {kernel_substr} in {d}")
    return sum(vals) / len(vals), len(vals)


def kernel_total_us(d: str, kernel_substr: str, exclude: tuple[str, ...] = ()) -> float:
    """Summed duration (us) of the dispatches of the kernels counter_per_dispatch selects."""
    return sum(calls * avg for name, calls, avg in kernel_times(d) if _match(name, kernel_substr, exclude))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--fetch-copy", required=True)
    ap.add_argument("--write-copy", required=True)
    ap.add_argument("--kernel", default="k_pass")
    ap.add_argument("--copy-kernel", default="copyBuffer")
    ap.add_argument("--out", required=True)
    ap.add_argument("--cmd", default="")
    ap.add_argument("--title", default="")
    ap.add_argument("--exclude", default="",
                    help="comma-separated name substrings of kernels to leave out of the selection")
    ap.add_argument("--units", type=int, default=0,
                    help="also report totals over all dispatches divided by this many units of work "
                         "(e.g. sorts), for kernels launched a varying number of times per unit")
    ap.add_argument("--unit-name", default="sort")
    ap.add_argument("--source", default=KERNEL_SRC,
                    help="kernel source file(s), comma-separated, whose joint hash is recorded")
    args = ap.parse_args()

    kt = kernel_times(args.trace)
    excl = tuple(x for x in args.exclude.split(",") if x)
    f_k, nf = counter_per_dispatch(args.fetch, "FETCH_SIZE", args.kernel, excl)
    w_k, nw = counter_per_dispatch(args.write, "WRITE_SIZE", args.kernel, excl)
    f_c, _ = counter_per_dispatch(args.fetch_copy, "FETCH_SIZE", args.copy_kernel)
    w_c, _ = counter_per_dispatch(args.write_copy, "WRITE_SIZE", args.copy_kernel)
    f_scale = COPY_BYTES / (f_c * 1024.0)
    w_scale = COPY_BYTES / (w_c * 1024.0)
    fetch_b = f_k * 1024.0 * f_scale
    write_b = w_k * 1024.0 * w_scale
    srcs = [x for x in args.source.split(",") if x]
    sha = hashlib.sha256(b"".join(open(x, "rb").read() for x in srcs)).hexdigest()[:16]
    dur = [t for t in kt if _match(t[0], args.kernel, excl)]
    lines = [f"# {args.title or args.kernel} rocprofv3 summary", ""]
    if args.cmd:
        lines += ["Commands (run from the repository root on an MI355X):", "", "```", args.cmd.strip(), "```", ""]
    lines += ["## Kernel durations (rocprofv3 --kernel-trace --stats)", "",
              "| kernel | calls | mean us |", "|---|---|---|"]
    for name, calls, avg in kt:
        lines.append(f"| {name.split('(')[0]} | {calls} | {avg:.2f} |")
    sel = f"`{args.kernel}`" + (f" except {', '.join('`' + x + '`' for x in excl)}" if excl else "")
    lines += ["", f"## HBM traffic of the kernels named {sel} (rocprofv3 --pmc, per dispatch)", "",
              f"- FETCH_SIZE mean over {nf} dispatches: {f_k:.1f} KiB (x{f_scale:.3f} copy calibration)",
              f"- WRITE_SIZE mean over {nw} dispatches: {w_k:.1f} KiB (x{w_scale:.3f} copy calibration)",
              f"- copy calibration: 256 MiB copy reads FETCH_SIZE {f_c:.1f} KiB, WRITE_SIZE {w_c:.1f} KiB", "",
              ]
    if args.units > 0:
        u = args.units
        lines += [f"Per {args.unit_name} ({u} in the run; totals over all {nf} dispatches / {u}):", "",
                  f"- kernel time: {kernel_total_us(args.trace, args.kernel, excl) / u:.2f} us",
                  f"- HBM fetch: {fetch_b * nf / u / 1e6:.2f} MB, write: {write_b * nw / u / 1e6:.2f} MB", ""]
    lines += ["Values read by bench.py:", "",
              f"kernel: {args.kernel}",
              f"mean_duration_us: {sum(t[2] * t[1] for t in dur) / max(sum(t[1] for t in dur), 1):.3f}",
              f"fetch_bytes_per_launch: {fetch_b:.0f}",
              f"write_bytes_per_launch: {write_b:.0f}",
              f"hbm_bytes_per_launch: {fetch_b + write_b:.0f}",
              "kernel_source: " + ",".join(os.path.relpath(x, os.path.dirname(HERE)) for x in srcs),
              f"kernel_source_sha: {sha}", ""]
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
