"""The C-ABI library loads and exports every entry point declared in include/*.h (CPU only: no
compute calls; argument errors are rejected on the host before anything touches a device)."""
from __future__ import annotations

import glob
import os
import re
import subprocess

import pytest

from paper_cs_0004013_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DECL = re.compile(r"^\s*(?:const\s+char\s*\*|ap_status|size_t|void)\s*\**\s*(ap_\w+)\s*\(", re.M)


def declared() -> list[str]:
    names = []
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        names += DECL.findall(open(h).read())
    return sorted(set(names))


def exported() -> set[str]:
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], check=True,
                         stdout=subprocess.PIPE, text=True).stdout
    return {line.split()[-1] for line in out.splitlines() if line.strip()}


@pytest.fixture(scope="module", autouse=True)
def built():
    from paper_cs_0004013_amd import build
    if build.is_stale():
        build.build()


def test_header_declares_entry_points():
    names = declared()
    for must in ("ap_sort_u32", "ap_sort_u32_ws", "ap_sort_workspace_bytes", "ap_digit_plan_u32",
                 "ap_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported():
    missing = [n for n in declared() if n not in exported()]
    assert not missing, missing


def test_library_loads_and_binds():
    L = binding.lib()
    for n in declared():
        assert hasattr(L, n)
    assert "gfx950" in binding.ap_version()


def test_workspace_size_is_host_only():
    L = binding.lib()
    assert L.ap_sort_workspace_bytes(1 << 30) == 0
    a, b = L.ap_sort_workspace_bytes(1 << 20), L.ap_sort_workspace_bytes(1 << 26)
    assert (1 << 22) < a < b and b >= 4 * (1 << 26)


def test_invalid_arguments_rejected_on_host():
    L = binding.lib()
    assert L.ap_sort_u32(None, None, 10, 64, None, None) == 1        # NULL buffers
    assert "NULL" in binding.last_error()
    assert L.ap_sort_u32(16, 32, 10, 0, None, None) == 1               # P < 1
    assert L.ap_sort_u32(16, 32, 1 << 30, 64, None, None) == 1         # n too large
    assert L.ap_sort_u32(18, 1024, 10, 64, None, None) == 1            # misaligned
    assert L.ap_sort_u32(4096, 4100, 10, 64, None, None) == 1          # partial overlap
    assert L.ap_digit_plan_u32(4096, 10, 3, 8192, None, None) == 1     # digit width
    assert L.ap_sort_u32_ws(4096, 8192, 1000, 4, None, 65536, 16, None) == 1  # workspace too small
    assert L.ap_merge_u32(4096, (1 << 64) - 1, 8192, 1, 65536, None) == 1   # na + nb wraps around
    assert L.ap_merge_u32(4096, 10, 8192, 10, 4100, None) == 1             # output overlaps a
    assert L.ap_merge_u32(None, 10, 8192, 10, 65536, None) == 1            # NULL run
    assert L.ap_merge_adjacent_u32(4096, 1 << 29, 1 << 29, None) == 1      # na + nb >= 2^30
    assert L.ap_merge_adjacent_u32(4098, 10, 10, None) == 1                # misaligned


def test_debug_pass_arguments():
    L = binding.lib()
    assert L.ap_debug_pass(3, 0, None, 0) == 1           # mode outside 0..2
    assert L.ap_debug_pass(-1, 0, None, 0) == 1
    assert L.ap_debug_pass(2, 0, None, 0) == 1           # trace mode without a buffer
    assert L.ap_debug_pass(2, 0, 4096, 0) == 1           # ... or without records
    assert L.ap_debug_pass(2, 0, 4100, 16) == 1          # misaligned buffer
    assert L.ap_debug_pass(1, 7, None, 0) == 0           # perturbation on, then off again
    assert L.ap_debug_pass(0, 0, None, 0) == 0
