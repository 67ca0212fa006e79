"""The oracle's pins are sharp: plausible mistakes planted in a copy of the oracle's C source
(on the CPU) make at least one pin fail.  Every planted mistake keeps memory accesses in bounds."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "apsort_oracle.c")

MUTANTS = {
    "drops lowest digit pass": ("for (int shift = 0; shift < 32;", "for (int shift = 8; shift < 32;"),
    "most significant digit first": (
        "for (int shift = 0; shift < 32; shift += ORACLE_DIGIT_BITS)",
        "for (int shift = 24; shift >= 0; shift -= ORACLE_DIGIT_BITS)"),
    "unstable partial sort (ties reversed)": (
        "for (size_t i = 0; i < n; ++i) {\n        unsigned v",
        "for (size_t i = n; i-- > 0;) {\n        unsigned v"),
    "partial sort writes the wrong element": ("dst[next[v]] = src[i];", "dst[next[v]] = src[n - 1 - i];"),
    "exclusive totals made inclusive-shifted": ("next[v] = running;\n        running += count[v];",
                                                "next[v] = running - (v ? count[v - 1] : 0);\n        running += count[v];"),
    "partial sort reads reversed digit": (
        "unsigned v = (src[i] >> shift) & (ORACLE_BUCKETS - 1);\n        dst",
        "unsigned v = (src[n - 1 - i] >> shift) & (ORACLE_BUCKETS - 1);\n        dst"),
    "upper cells take the extra element": ("pos += q + ((uint64_t)p < r ? 1 : 0);",
                                           "pos += q + ((uint64_t)(P - 1 - p) < r ? 1 : 0);"),
    "splitter is last key of the lower cell": ("? sorted[starts[p]] :", "? sorted[starts[p] - 1] :"),
    "histogram digit off by one bit": ("hist[(keys[i] >> shift) & mask] += 1;",
                                       "hist[(keys[i] >> (shift + 1)) & mask] += 1;"),
    "empty cell not padded": (": 0xFFFFFFFFu;", ": 0u;"),
    "pairs: value left in place": ("dst_v[slot] = src_v[j];", "dst_v[j] = src_v[j];"),
    "pairs: value of the mirrored element": ("dst_v[slot] = src_v[j];", "dst_v[slot] = src_v[n - 1 - j];"),
    "pairs: ties reversed": ("    for (size_t j = 0; j < n; ++j) {\n        unsigned b",
                             "    for (size_t j = n; j-- > 0;) {\n        unsigned b"),
    "pairs: only three digit passes": ("for (int d = 0; d < 4; ++d)", "for (int d = 0; d < 3; ++d)"),
    "merge: rest of the second list dropped": ("    while (j < nb)\n        out[k++] = b[j++];", "    while (j + 1 < nb)\n        out[k++] = b[j++];"),
    "merge: compares against the previous head": ("if (b[j] < a[i])", "if (j > 0 && b[j - 1] < a[i])"),
    "merge: takes the larger head": ("if (b[j] < a[i])", "if (b[j] > a[i])"),
    "mt: totals taken thread by thread": (
        "for (unsigned v = 0; v < ORACLE_BUCKETS; ++v)\n            for (int t = 0; t < nthreads; ++t) {",
        "for (int t = 0; t < nthreads; ++t)\n            for (unsigned v = 0; v < ORACLE_BUCKETS; ++v) {"),
    "mt: a thread moves its chunk backwards": (
        "for (size_t i = j->lo; i < j->hi; ++i) {\n        unsigned v",
        "for (size_t i = j->hi; i-- > j->lo;) {\n        unsigned v"),
}


def _battery() -> bool:
    """Run the pins; True when all of them hold."""
    try:
        pins.test_golden_lsd_trace()
        for n, P, sizes in pins._read_slices():
            pins.test_golden_cell_sizes(n, P, sizes)
        for n in (0, 5, 300, 4096, 70001):
            pins.test_vs_numpy_sort(n)
        pins.test_exhaustive_tiny_domain()
        for shift in (0, 8, 16, 24):
            pins.test_bucket_pass_is_stable_digit_sort(shift)
        for shift, bits in ((0, 8), (8, 8), (24, 8), (0, 11)):
            pins.test_digit_hist_vs_bincount(shift, bits)
        for n in (1, 5, 1000):
            pins.test_closed_forms(n)
        pins.test_segmented_vs_per_segment_numpy()
        pins.test_pairs_exhaustive_tiny_domain()
        for dist in ("a", "c", "e"):
            pins.test_pairs_values_are_stable_argsort(dist)
        for shift in (0, 16):
            pins.test_pairs_bucket_pass_is_stable_digit_sort(shift)
        pins.test_pairs_keys_match_key_sort()
        pins.test_merge_exhaustive_tiny_domain()
        for na, nb in ((1000, 3), (70_001, 65_536)):
            pins.test_merge_vs_numpy(na, nb)
        pins.test_merge_closed_forms()
        for n, threads in ((300, 3), (70_001, 8), (5, 16)):
            pins.test_mt_variant_vs_numpy_and_single_thread(n, threads)
    except AssertionError:
        return False
    return True


def _compile(src_text: str, out_dir: str, name: str) -> str:
    c = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-pthread", "-o", so, c])
    return so


def test_unmutated_passes(tmp_path, monkeypatch):
    so = _compile(open(SRC).read(), str(tmp_path), "orig")
    monkeypatch.setattr(oracle, "_lib", oracle._bind(so))
    assert _battery()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not found for {name!r}"
    so = _compile(text.replace(old, new), str(tmp_path), "mut")
    monkeypatch.setattr(oracle, "_lib", oracle._bind(so))
    assert not _battery(), f"no pin caught: {name}"
