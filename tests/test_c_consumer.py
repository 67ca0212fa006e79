"""The C ABI used from plain C: tests/c/consumer.c (device memory from the HIP runtime's C API,
every sort through include/apsort.h) must compile as C11 against the header, link against
libapsort.so, and, on a GPU, sort one array, one array in place with a caller workspace, a
segmented batch and three served requests exactly (checked against qsort inside the program)."""
from __future__ import annotations

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_cs_0004013_amd")
SRC = os.path.join(ROOT, "tests", "c", "consumer.c")


def _build(out: str) -> None:
    if not os.path.exists(os.path.join(PKG, "libapsort.so")):
        pytest.skip("libapsort.so is not built")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), SRC, "-L" + PKG, "-lapsort", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath," + PKG, "-Wl,-rpath,/opt/rocm/lib", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr


def test_c_consumer_compiles_and_links(tmp_path):
    _build(str(tmp_path / "consumer"))


@pytest.mark.gpu
def test_c_consumer_runs(tmp_path):
    exe = str(tmp_path / "consumer")
    _build(exe)
    print("running the C consumer", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "consumer ok" in r.stdout
