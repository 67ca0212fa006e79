"""Length-group table of the segmented sort: the used groups must cover every length class 1..31
exactly once (CPU only: the checks run on the host before anything touches a device)."""
from __future__ import annotations

import os

import pytest

from paper_cs_0004013_amd import binding


@pytest.fixture(scope="module", autouse=True)
def built():
    from paper_cs_0004013_amd import build
    if build.is_stale():
        build.build()


@pytest.fixture
def saved_groups():
    saved = binding.segmented_groups()
    yield
    binding.set_segmented_groups(saved)


def _table(tmp_path, rows) -> str:
    p = os.path.join(tmp_path, "tune.txt")
    with open(p, "w") as f:
        f.write("# test table\n")
        for g, (lo, hi, cfg) in enumerate(rows):
            f.write(f"{g} {lo} {hi} {cfg}\n")
    return p


def test_installed_table_is_a_partition(saved_groups):
    owner = {}
    for g, (lo, hi, _cfg) in enumerate(binding.segmented_groups()):
        for c in range(lo, hi + 1):
            assert c not in owner, (c, owner[c], g)
            owner[c] = g
    assert sorted(owner) == list(range(1, 32))


def test_load_tuning_rejects_overlap(tmp_path, saved_groups):
    before = binding.segmented_groups()
    p = _table(str(tmp_path), [(14, 31, 10), (12, 14, 1), (1, 11, 3)])   # class 14 twice
    with pytest.raises(binding.ApError) as e:
        binding.ap_load_tuning(p)
    assert e.value.status == 1 and "both cover length class 14" in str(e.value)
    assert binding.segmented_groups() == before                         # nothing installed


def test_load_tuning_rejects_gap(tmp_path, saved_groups):
    before = binding.segmented_groups()
    p = _table(str(tmp_path), [(14, 31, 10), (1, 12, 3)])                # class 13 uncovered
    with pytest.raises(binding.ApError) as e:
        binding.ap_load_tuning(p)
    assert e.value.status == 1 and "no length group covers length class 13" in str(e.value)
    assert binding.segmented_groups() == before


def test_load_tuning_accepts_partition(tmp_path, saved_groups):
    rows = [(15, 31, 1), (12, 14, 5), (9, 11, 2), (1, 8, 4)]
    binding.ap_load_tuning(_table(str(tmp_path), rows))
    got = binding.segmented_groups()
    assert got[:4] == rows and all(lo > hi for lo, hi, _ in got[4:])


@pytest.mark.parametrize("rows, msg", [
    ([(14, 31, 10), (13, 14, 1), (12, 12, 5), (1, 11, 3)], "both cover length class 14"),
    ([(14, 31, 10), (12, 12, 5), (1, 11, 3)], "no length group covers length class 13"),
])
def test_segmented_call_rejects_bad_table(rows, msg, saved_groups):
    """A table built group by group is checked when the sort is called: AP_ERR_INVALID, with
    nothing enqueued (the pointers below are never dereferenced)."""
    binding.set_segmented_groups(rows)
    L = binding.lib()
    assert L.ap_sort_u32_segmented(4096, 1000, 8192, 4, None, None) == 1
    assert msg in binding.last_error()
