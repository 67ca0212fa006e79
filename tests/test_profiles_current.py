"""The committed rocprofv3 summaries under profiles/ were taken on the kernel sources as they are
now: each summary that names its sources carries their hash, and it must match (a stale summary
would make the bench drop the measured traffic and would describe a kernel that no longer exists)."""
from __future__ import annotations

import glob
import hashlib
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUMMARIES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))


def _fields(path: str) -> dict:
    out = {}
    for line in open(path):
        line = line.strip()
        for key in ("kernel_source", "kernel_source_sha"):
            if line.startswith(key + ":"):
                out[key] = line.partition(":")[2].strip()
    return out


@pytest.mark.parametrize("path", SUMMARIES, ids=[os.path.basename(p) for p in SUMMARIES])
def test_summary_matches_sources(path):
    f = _fields(path)
    if "kernel_source_sha" not in f:
        pytest.skip("summary names no source hash")
    srcs = [os.path.join(ROOT, s) for s in f["kernel_source"].split(",")]
    sha = hashlib.sha256(b"".join(open(s, "rb").read() for s in srcs)).hexdigest()[:16]
    assert sha == f["kernel_source_sha"], f"{os.path.basename(path)} was taken on other sources"


def test_bench_reads_the_k_pass_summary():
    import bench
    prof = bench.read_profile()
    assert prof is not None and prof["traffic"] > 0 and prof["mean_us"] > 0
