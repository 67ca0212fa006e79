"""Parity of the bucketing variant (ap_sort_u32_msd: order by the top 16 bits, then a local sort of
every bucket) with the CPU oracle, element by element, through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_cs_0004013_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _msd(keys: np.ndarray, P: int = 64, inplace: bool = False):
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    t_in, _ = to_dev(keys)
    t_out = t_in if inplace else torch.full_like(t_in, 0x5151)
    spl = torch.full((max(P - 1, 1),), 0x1111, dtype=torch.int32, device="cuda")
    binding.ap_sort_u32_msd(t_in, t_out, P, spl if P > 1 else None)
    torch.cuda.synchronize()
    return to_host(t_out), to_host(spl)[:max(P - 1, 0)]


def _check(keys, P=64, **kw):
    announce(f"msd n={keys.size} P={P} {kw}")
    got, spl = _msd(keys, P, **kw)
    want = oracle.sort_u32(keys)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    assert np.array_equal(spl, oracle.splitters(want, P))


@pytest.mark.parametrize("dist", inputs.DISTS)
def test_distributions_2pow22(dist):
    _check(inputs.keyset(dist, (1 << 22) + 5, seed=13).keys)


@pytest.mark.parametrize("seed,dist", [(1, "a"), (5, "e")])
def test_distributions_full_size(seed, dist):
    """2^26 keys, the benchmark's (a) and (e) workloads."""
    _check(inputs.keyset(dist, 1 << 26, seed=seed).keys)


def test_adversarial():
    """Top 16 bits take 4 values: four buckets of ~2^25 keys go through the device-wide passes."""
    _check(inputs.adversarial(1 << 27, seed=0).keys)


@pytest.mark.parametrize("n", [1, 2, 3, 64, 65, 1000, 65_537, (1 << 20) + 3])
def test_sizes_full_range_keys(n):
    rng = np.random.default_rng(n + 1)
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    _check(keys)
    _check(keys, P=n + 1)


def test_in_place_and_closed_forms():
    rng = np.random.default_rng(2)
    n = (1 << 21) + 9
    _check(rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32), inplace=True)
    perm = rng.permutation(n).astype(np.uint32)
    got, _ = _msd(perm, 7)
    assert np.array_equal(got, np.arange(n, dtype=np.uint32))
    _check(np.full(n, 0x80000001, np.uint32), inplace=True)      # one bucket, every digit constant
    _check(rng.integers(0, 1 << 16, size=n, dtype=np.uint64).astype(np.uint32))   # top 16 bits constant


def test_empty_and_repeat():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    spl = torch.zeros(7, dtype=torch.int32, device="cuda")
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    binding.ap_sort_u32_msd(e, e, 8, spl)
    torch.cuda.synchronize()
    assert (to_host(spl) == 0xFFFFFFFF).all()
    keys = inputs.keyset("d", 300_001, seed=3).keys
    t_in, _ = to_dev(keys)
    t_out = torch.empty_like(t_in)
    for _ in range(3):                      # the segmented graph is captured, then replayed
        binding.ap_sort_u32_msd(t_in, t_out, 64, None)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(t_out), oracle.sort_u32(keys))
