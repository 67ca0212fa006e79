"""The digit pass under its debug modes (ap_debug_pass), through the C ABI.

Mode 1 perturbs the timing of every tile with seeded delays at the claim and before the scan, the
reorder, the look-back, the inclusive prefix and the scatter (Sec. 3.2 distribution of one digit,
with the per-tile bucket totals combined by the look-back): tiles then publish and finish in
orders the normal timing seldom gives.  The results must stay bit-exact against the oracle.
Mode 2 records per-tile phase timestamps; the records must be complete and ordered, and the sort
still exact.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_cs_0004013_amd import inputs
from tests.gpu_util import announce, gpu_sort, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture
def debug_off():
    from paper_cs_0004013_amd import binding
    yield binding
    binding.ap_debug_pass(0)
    binding.ap_set_rank_mode(0)
    binding.ap_set_pass_shape(-1)


def _exact(keys: np.ndarray, P: int = 64):
    out, spl = gpu_sort(keys, P)
    want = oracle.sort_u32(keys)
    bad = np.flatnonzero(out != want)
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    assert np.array_equal(spl, oracle.splitters(want, P))


# sizes across the four tile shapes by size (4K, 8K, 16K and 32K keys), each with a ragged last tile
@pytest.mark.parametrize("n", [(1 << 16) + 77, (1 << 19) + 5, (1 << 21) + 3, (1 << 25) + 1001])
@pytest.mark.parametrize("seed", [1, 2])
def test_perturbed_uniform(debug_off, n, seed):
    torch_cuda()
    debug_off.ap_debug_pass(1, seed)
    announce(f"perturbed pass n={n} seed={seed}")
    _exact(inputs.keyset("a", n, seed=seed).keys)


@pytest.mark.parametrize("dist", ["b", "d", "e"])
def test_perturbed_distributions(debug_off, dist):
    torch_cuda()
    debug_off.ap_debug_pass(1, 11)
    announce(f"perturbed pass dist={dist}")
    _exact(inputs.keyset(dist, (1 << 24) + 9, seed=5).keys)


def test_perturbed_adversarial(debug_off):
    torch_cuda()
    debug_off.ap_debug_pass(1, 3)
    announce("perturbed pass adversarial 2^23")
    _exact(inputs.adversarial((1 << 23) + 1, seed=3).keys)


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_perturbed_mask_rank(debug_off, shape):
    torch_cuda()
    debug_off.ap_set_rank_mode(1)
    debug_off.ap_set_pass_shape(shape)
    debug_off.ap_debug_pass(1, 17 + shape)
    announce(f"perturbed pass, mask rank, shape {shape}")
    _exact(inputs.keyset("a", (1 << 22) + 31, seed=shape).keys)


def test_phase_trace(debug_off):
    torch = torch_cuda()
    b = debug_off
    n = (1 << 24) + 5
    keys = inputs.keyset("a", n, seed=4).keys
    tile = 16 * 64 * 32 if n >= (1 << 22) else 16 * 64 * 16   # the shape chosen by size
    ntiles = (n + tile - 1) // tile
    trace = torch.zeros((4 * ntiles + 16) * b.PASS_TRACE_WORDS, dtype=torch.int64, device="cuda")
    b.ap_debug_pass(2, 0, trace)
    announce(f"phase trace n={n} tiles={ntiles}")
    _exact(keys)
    rec = trace.cpu().numpy().reshape(-1, b.PASS_TRACE_WORDS)
    used = rec[:4 * ntiles, :6]
    assert np.all(used > 0), "a tile of a pass left no record"
    assert np.all(np.diff(used, axis=1) >= 0), "phase timestamps out of order"
    assert np.all(rec[4 * ntiles:] == 0), "records written past the last tile"
    # passes run one after another on the stream
    ends = used[:, 5].reshape(4, ntiles).max(axis=1)
    starts = used[:, 0].reshape(4, ntiles).min(axis=1)
    assert np.all(starts[1:] >= ends[:-1])
