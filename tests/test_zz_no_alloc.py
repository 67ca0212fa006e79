"""ap_sort_u32_noalloc (scratch in the library's fixed device array, no allocation) gives exactly
the results of ap_sort_u32 through the C ABI, on consecutive calls that share the array (the
second one smaller), and rejects sizes beyond its maximum."""
from __future__ import annotations

import numpy as np
import pytest

from paper_cs_0004013_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _both(keys: np.ndarray, P: int, inplace: bool = False):
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    t_in, _ = to_dev(keys)
    ref = torch.empty_like(t_in)
    spl_ref = torch.full((max(P - 1, 1),), 0x2222, dtype=torch.int32, device="cuda")
    binding.ap_sort_u32(t_in, ref, P, spl_ref if P > 1 else None)
    t_in2, _ = to_dev(keys)
    out = t_in2 if inplace else torch.full_like(t_in2, 0x3333)
    spl = torch.full((max(P - 1, 1),), 0x4444, dtype=torch.int32, device="cuda")
    binding.ap_sort_u32_noalloc(t_in2, out, P, spl if P > 1 else None)
    torch.cuda.synchronize()
    return (to_host(ref), to_host(spl_ref)[:P - 1]), (to_host(out), to_host(spl)[:P - 1])


@pytest.mark.parametrize("sizes", [((1 << 22), 5000), ((1 << 20) + 77, 3), (300_001, 300_000)])
def test_two_calls_in_a_row_match_plain_sort(sizes):
    for i, n in enumerate(sizes):
        keys = inputs.keyset("ae"[i % 2], n, seed=60 + i).keys
        announce(f"noalloc call {i} n={n}")
        (ref, spl_ref), (got, spl) = _both(keys, 64)
        assert np.array_equal(got, ref), f"call {i}"
        assert np.array_equal(spl, spl_ref), f"call {i} splitters"


def test_in_place_and_degenerate_inputs():
    rng = np.random.default_rng(61)
    for keys in (rng.integers(0, 1 << 32, size=70_001, dtype=np.uint64).astype(np.uint32),
                 np.full(9000, 5, np.uint32), np.arange(3, dtype=np.uint32)[::-1].copy()):
        (ref, spl_ref), (got, spl) = _both(keys, 7, inplace=True)
        assert np.array_equal(got, ref) and np.array_equal(spl, spl_ref)


def test_rejects_beyond_maximum():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    n = binding.NOALLOC_MAX_KEYS + 1
    t = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.ApError) as e:
        binding.ap_sort_u32_noalloc(t, t, 64)
    assert e.value.status == 1 and "no-allocation maximum" in str(e.value)
