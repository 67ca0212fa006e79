"""The profile summary tool on small hand-made rocprofv3 databases: per-dispatch means, copy
calibration, the --exclude selection and the per-unit totals."""
from __future__ import annotations

import os
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _trace_db(d, rows):
    os.makedirs(d)
    con = sqlite3.connect(os.path.join(d, "run_results.db"))
    con.execute("create table top_kernels (name text, total_calls int, average real)")
    con.executemany("insert into top_kernels values (?, ?, ?)", rows)
    con.commit()


def _pmc_db(d, counter, rows):
    os.makedirs(d)
    con = sqlite3.connect(os.path.join(d, "run_results.db"))
    con.execute("create table counters_collection (kernel_name text, dispatch_id int, counter_name text, value real)")
    # each dispatch's value split over two instances, as rocprofv3 records one row per instance
    con.executemany("insert into counters_collection values (?, ?, ?, ?)",
                    [(k, i, counter, v / 2) for k, i, v in rows for _ in range(2)])
    con.commit()


def test_summary_values(tmp_path):
    t = str(tmp_path)
    _trace_db(f"{t}/trace", [("void aps::k_pass<8>(x)", 4, 100.0), ("aps::k_finalize(y)", 2, 5.0),
                             ("aps::k_check_one(z)", 1, 50.0)])
    # k_pass: two real passes (1000 / 3000 KiB read) and two that exit at once (0 KiB)
    _pmc_db(f"{t}/fetch", "FETCH_SIZE", [("void aps::k_pass<8>(x)", 1, 1000.0), ("void aps::k_pass<8>(x)", 2, 3000.0),
                                         ("void aps::k_pass<8>(x)", 3, 0.0), ("void aps::k_pass<8>(x)", 4, 0.0),
                                         ("aps::k_finalize(y)", 5, 10.0), ("aps::k_check_one(z)", 6, 9999.0)])
    _pmc_db(f"{t}/write", "WRITE_SIZE", [("void aps::k_pass<8>(x)", 1, 2000.0), ("void aps::k_pass<8>(x)", 2, 2000.0),
                                         ("void aps::k_pass<8>(x)", 3, 0.0), ("void aps::k_pass<8>(x)", 4, 0.0),
                                         ("aps::k_finalize(y)", 5, 20.0), ("aps::k_check_one(z)", 6, 0.0)])
    # a 256 MiB copy that reads half its bytes on FETCH_SIZE and all on WRITE_SIZE
    _pmc_db(f"{t}/fc", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 1, 131072.0)])
    _pmc_db(f"{t}/wc", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 1, 262144.0)])
    out = f"{t}/s.md"
    cmd = [sys.executable, "-m", "paper_cs_0004013_amd.profile_summary", "--trace", f"{t}/trace", "--fetch",
           f"{t}/fetch", "--write", f"{t}/write", "--fetch-copy", f"{t}/fc", "--write-copy", f"{t}/wc",
           "--out", out]
    subprocess.run(cmd + ["--kernel", "k_pass", "--units", "2"], check=True, cwd=ROOT, capture_output=True)
    txt = open(out).read()
    vals = dict(l.split(": ", 1) for l in txt.splitlines() if ": " in l and not l.startswith(("-", "#", "|")))
    assert vals["kernel"] == "k_pass"
    assert float(vals["mean_duration_us"]) == 100.0
    assert int(vals["fetch_bytes_per_launch"]) == 1000 * 1024 * 2   # mean 1000 KiB x2 calibration
    assert int(vals["write_bytes_per_launch"]) == 1000 * 1024
    # per unit: all four dispatches over two units
    assert "kernel time: 200.00 us" in txt
    assert f"HBM fetch: {4 * 1000 * 1024 * 2 / 2 / 1e6:.2f} MB, write: {4 * 1000 * 1024 / 2 / 1e6:.2f} MB" in txt
    # every aps kernel but the check
    subprocess.run(cmd + ["--kernel", "aps::k_", "--exclude", "k_check", "--units", "1"], check=True, cwd=ROOT,
                   capture_output=True)
    txt = open(out).read()
    assert "kernel time: 410.00 us" in txt
    assert f"HBM fetch: {4010 * 1024 * 2 / 1e6:.2f} MB, write: {4020 * 1024 / 1e6:.2f} MB" in txt
    assert "except `k_check`" in txt
