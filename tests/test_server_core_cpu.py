"""Scheduling core of the request server on the CPU: builds tests/cpp/test_server_core.cpp (host code
only) against the core header and the CPU oracle, plain, with ThreadSanitizer and with
AddressSanitizer + UndefinedBehaviorSanitizer, and runs it.

ThreadSanitizer uses ROCm's clang: the GCC 11 runtime does not intercept pthread_cond_clockwait
(used by std::condition_variable::wait_for) and then reports false races on every timed wait."""
from __future__ import annotations

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


CLANG = "/opt/rocm/llvm/bin/clang"


def _build_and_run(tmp_path, sanitize: str | None, cc: str = "gcc", cxx: str = "g++"):
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "server_core_test")
    subprocess.check_call([cc, "-O1", "-g", "-c", "-fPIC", os.path.join(ROOT, "oracle", "apsort_oracle.c"),
                           "-o", obj] + ([f"-fsanitize={sanitize}"] if sanitize else []))
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_cs_0004013_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "test_server_core.cpp"), obj, "-o", exe, "-lpthread"]
    if sanitize:
        cmd.insert(1, f"-fsanitize={sanitize}")
    subprocess.check_call(cmd)
    res = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    assert res.returncode == 0 and "ALL PASSED" in res.stdout, res.stdout[-4000:]


def test_server_core_plain(tmp_path):
    _build_and_run(tmp_path, None)


def test_server_core_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, "thread", CLANG, CLANG + "++")


def test_server_core_address_ub_sanitizer(tmp_path):
    _build_and_run(tmp_path, "address,undefined")
