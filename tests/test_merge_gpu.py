"""Parity of the merge of two sorted runs (merge-exchange merge step) with the CPU oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_cs_0004013_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _runs(na: int, nb: int, seed: int, dom: int = 1 << 32):
    rng = np.random.default_rng(seed)
    a = np.sort(rng.integers(0, dom, size=na, dtype=np.uint64).astype(np.uint32))
    b = np.sort(rng.integers(0, dom, size=nb, dtype=np.uint64).astype(np.uint32))
    return a, b


def _merge(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    announce(f"merge na={a.size} nb={b.size}")
    ta, _ = to_dev(a)
    tb, _ = to_dev(b)
    out, _ = to_dev(np.zeros(a.size + b.size, np.uint32))
    binding.ap_merge_u32(ta, tb, out)
    torch.cuda.synchronize()
    return to_host(out)


@pytest.mark.parametrize("na,nb", [(0, 1), (1, 0), (1, 1), (4095, 1), (4096, 4096), (4097, 5000), (70_001, 3),
                                   (3, 70_001), ((1 << 20) + 17, (1 << 19) - 5)])
def test_sizes(na, nb):
    a, b = _runs(na, nb, na + nb)
    assert np.array_equal(_merge(a, b), oracle.merge_u32(a, b))


@pytest.mark.parametrize("dom", [1, 3, 1000])
def test_many_equal_keys(dom):
    a, b = _runs(300_007, 250_001, dom, dom)
    assert np.array_equal(_merge(a, b), oracle.merge_u32(a, b))


def test_disjoint_ranges():
    lo = np.arange(100_000, dtype=np.uint32)
    hi = np.arange(100_000, 180_000, dtype=np.uint32)
    assert np.array_equal(_merge(hi, lo), oracle.merge_u32(hi, lo))
    assert np.array_equal(_merge(lo, hi), oracle.merge_u32(lo, hi))


def test_full_size_halves():
    """Two sorted halves of the 2^26-key uniform workload."""
    keys = inputs.keyset("a", 1 << 26, seed=1).keys
    a = np.sort(keys[: 1 << 25])
    b = np.sort(keys[1 << 25:])
    assert np.array_equal(_merge(a, b), oracle.merge_u32(a, b))


@pytest.mark.parametrize("na,nb", [(1, 1), (5000, 0), (123_457, 98_765)])
def test_adjacent_in_place(na, nb):
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    a, b = _runs(na, nb, 77, 1 << 20)
    t, _ = to_dev(np.concatenate([a, b]))
    binding.ap_merge_adjacent_u32(t, na)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(t), oracle.merge_u32(a, b))


def test_overlapping_output_rejected():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    x = torch.zeros(3000, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.ApError):
        binding.ap_merge_u32(x[:1000], x[1000:2000], x[500:2500])


def test_maximum_size():
    """na + nb = 2^30 - 1 (the largest total accepted), runs of 31-bit keys (signed and unsigned
    order agree), against torch's sort of the concatenation on the device; then the same runs as
    one array through the adjacent-run merge."""
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    na, nb = 1 << 29, (1 << 29) - 1
    announce(f"merge maximum size na={na} nb={nb}")
    g = torch.Generator(device="cuda").manual_seed(6)
    keys = torch.randint(0, 1 << 31, (na + nb,), device="cuda", generator=g, dtype=torch.int32)
    keys[::7] &= 0xFF                                   # ties across the two runs
    a = torch.sort(keys[:na])[0]
    b = torch.sort(keys[na:])[0]
    want = torch.sort(keys)[0]
    del keys
    out = torch.empty(na + nb, dtype=torch.int32, device="cuda")
    binding.ap_merge_u32(a, b, out)
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    out[:na] = a
    out[na:] = b
    del a, b
    binding.ap_merge_adjacent_u32(out, na)
    torch.cuda.synchronize()
    assert torch.equal(out, want)


def test_release_cache_between_merges():
    """ap_release_cache frees the merge scratch too: merges before and after it (each one after a
    release re-allocates) all match the oracle."""
    from paper_cs_0004013_amd import binding
    a, b = _runs(70_001, 65_536, 5)
    assert np.array_equal(_merge(a, b), oracle.merge_u32(a, b))
    binding.ap_release_cache()
    a2, b2 = _runs(300_000, 123_457, 6)
    assert np.array_equal(_merge(a2, b2), oracle.merge_u32(a2, b2))
    binding.ap_release_cache()
    assert np.array_equal(_merge(a, b), oracle.merge_u32(a, b))
