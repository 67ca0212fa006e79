"""The device result check (ap_check_u32) against the same quantities computed in numpy: the number
of descents of the sequence and the SplitMix64 sum/xor multiset hash of tests/invariants.py."""
from __future__ import annotations

import numpy as np
import pytest

from paper_cs_0004013_amd import inputs
from tests import invariants as inv
from tests.gpu_util import announce, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _device_check(keys: np.ndarray, pad_front: int = 0):
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    t, _ = to_dev(keys, pad_front)
    acc = torch.zeros(3, dtype=torch.int64, device="cuda")
    binding.ap_check_u32(t, acc)
    torch.cuda.synchronize()
    a = acc.cpu().numpy().view(np.uint64)
    return int(a[0]), int(a[1]), int(a[2])


@pytest.mark.parametrize("n", [0, 1, 2, 3, 255, 4097, 1 << 20, (1 << 22) + 5])
def test_matches_numpy(n):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    announce(f"check n={n}")
    bad, s, x = _device_check(keys, pad_front=n % 3)
    assert bad == int(np.count_nonzero(keys[:-1] > keys[1:])) if n > 1 else bad == 0
    assert (s, x) == inv.multiset_hash(keys)
    srt = np.sort(keys)
    bad2, s2, x2 = _device_check(srt)
    assert bad2 == 0 and (s2, x2) == (s, x)


def test_batch_form_matches_single_calls():
    """ap_check_u32_batch over arrays of mixed lengths (0, ragged, large) gives, per array, what
    the single-array call gives, with max_n both exact and too small."""
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    rng = np.random.default_rng(7)
    lens = [0, 1, 2, 777, 4096, 300_001, 5, 1 << 20]
    arrs = [rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32) for n in lens]
    for i in (2, 4):
        arrs[i] = np.sort(arrs[i])
    devs = [to_dev(a)[0] for a in arrs]
    ptrs = torch.tensor([t.data_ptr() for t in devs], dtype=torch.int64, device="cuda")
    cnts = torch.tensor(lens, dtype=torch.int64, device="cuda")
    for max_n in (max(lens), 1000):
        acc = torch.zeros((len(lens), 3), dtype=torch.int64, device="cuda")
        binding.ap_check_u32_batch(ptrs.data_ptr(), cnts.data_ptr(), len(lens), max_n, acc.data_ptr())
        torch.cuda.synchronize()
        got = acc.cpu().numpy().view(np.uint64)
        for a, row in zip(arrs, got):
            assert tuple(int(v) for v in row) == _device_check(a)


def test_detects_one_changed_key():
    keys = np.sort(inputs.keyset("d", 100_000, seed=3).keys)
    ref = _device_check(keys)
    wrong = keys.copy()
    i = 5000 + int(np.flatnonzero(np.diff(keys[5000:].astype(np.int64)) >= 2)[0])
    wrong[i] += np.uint32(1)                     # still sorted, different multiset
    got = _device_check(wrong)
    assert got[0] == 0 and got[1:] != ref[1:]
    swapped = keys.copy()
    swapped[[10, 90_000]] = swapped[[90_000, 10]]  # same multiset, not sorted
    got = _device_check(swapped)
    assert got[0] > 0 and got[1:] == ref[1:]
