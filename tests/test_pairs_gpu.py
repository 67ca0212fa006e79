"""Parity of the (key, value) pairs sort with the CPU oracle, through the C ABI.

The oracle's pairs sort is stable (equal keys keep their input order), so with values equal to
input positions the expected values are the unique stable sorting permutation: the comparison
is bit-exact for keys, values and splitters."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_cs_0004013_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _pairs(keys: np.ndarray, vals: np.ndarray, P: int = 64, inplace: bool = False):
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    announce(f"pairs n={keys.size} P={P} inplace={inplace}")
    k_in, _kb = to_dev(keys)
    v_in, _vb = to_dev(vals)
    if inplace:
        k_out, v_out = k_in, v_in
    else:
        k_out, _ = to_dev(np.zeros(keys.size, np.uint32))
        v_out, _ = to_dev(np.zeros(keys.size, np.uint32))
    spl = torch.empty(max(P - 1, 1), dtype=torch.int32, device="cuda")
    binding.ap_sort_pairs_u32(k_in, v_in, k_out, v_out, P, spl)
    torch.cuda.synchronize()
    return to_host(k_out), to_host(v_out), to_host(spl)[:max(P - 1, 0)]


def _check(keys: np.ndarray, vals: np.ndarray | None = None, P: int = 64, inplace: bool = False):
    if vals is None:
        vals = np.arange(keys.size, dtype=np.uint32)
    gk, gv, gs = _pairs(keys, vals, P, inplace)
    wk, wv = oracle.sort_pairs_u32(keys, vals)
    bad = np.flatnonzero((gk != wk) | (gv != wv))
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    assert np.array_equal(gs, oracle.splitters(wk, P))


# around the pairs' tile thresholds by size (2^17: 4K -> 8K keys; 2^22: 8K -> 16K keys)
@pytest.mark.parametrize("n", [1, 2, 5, 63, 2047, 2048, 2049, 70_001, (1 << 17) - 1, 1 << 17, (1 << 20) + 7,
                               (1 << 22) - 1, (1 << 22) + 77])
def test_sizes(n):
    _check(inputs.keyset("e", n, seed=n % 97).keys)


# the pairs pass loads with the non-temporal hint from 2^24 to 5*2^23 pairs and plainly outside:
# both sides of both boundaries, with the atomic rank (16 x 16 tile) and the mask rank (8 x 32)
@pytest.mark.parametrize("rank_mode", [0, 1])
@pytest.mark.parametrize("n", [(1 << 24) - 1, 1 << 24, 5 << 23, (5 << 23) + 1])
def test_load_hint_boundaries(n, rank_mode):
    from paper_cs_0004013_amd import binding
    binding.ap_set_rank_mode(rank_mode)
    try:
        _check(inputs.keyset("d", n, seed=n % 89 + rank_mode).keys)
    finally:
        binding.ap_set_rank_mode(0)


@pytest.mark.parametrize("dist", inputs.DISTS)
def test_distributions_with_payload(dist):
    ks = inputs.keyset(dist, (1 << 21) + 333, seed=17)
    pos = np.arange(ks.keys.size, dtype=np.uint32)
    _check(ks.keys, (pos * np.uint32(2654435761)) ^ np.uint32(0xC2B2AE35))


def test_full_size_clustered_keys():
    """2^26 keys of distribution (e): at most ~4096 distinct values, so nearly every key has
    thousands of equal keys and the stable order of their values is fully observable."""
    _check(inputs.keyset("e", 1 << 26, seed=5).keys)


@pytest.mark.parametrize("seed", [0, 1])
def test_runs_of_equal_keys(seed):
    """Runs of equal keys of random lengths 1..199 in input order: one wave's rank slots switch
    between all-lanes-equal digits (one add of 64) and mixed digits (lane-ordered atomics), in
    every pass; the values (input positions) must come out as the stable argsort."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(1, 200, size=30_000)
    vals = rng.integers(0, 1 << 32, size=lens.size, dtype=np.uint64).astype(np.uint32)
    vals[::3] &= np.uint32(0xFF)              # some runs differ only in the low digit
    keys = np.repeat(vals, lens)
    _check(keys)


def test_maximum_size():
    """n = 2^30 - 1 pairs (the largest n accepted), values 0..n-1, checked on the device by
    properties that fix the stable sort uniquely: keys nondecreasing (unsigned), every output key
    equal to the input key at its output value, and values increasing within runs of equal keys
    (the values are then a permutation: a gather of n distinct positions in increasing order per
    key)."""
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    n = (1 << 30) - 1
    announce(f"pairs maximum size n={n}")
    g = torch.Generator(device="cuda").manual_seed(3)
    keys = torch.randint(-(1 << 31), 1 << 31, (n,), device="cuda", generator=g, dtype=torch.int32)
    keys[: n // 2] &= 0xFFFF                      # half the keys from 2^16 values: long runs of ties
    vals = torch.arange(n, device="cuda", dtype=torch.int32)
    ko = torch.empty_like(keys)
    vo = torch.empty_like(vals)
    binding.ap_sort_pairs_u32(keys, vals, ko, vo, 64, None)
    torch.cuda.synchronize()
    flip = ko ^ torch.tensor(-(1 << 31), dtype=torch.int32, device="cuda")
    assert bool((flip[1:] >= flip[:-1]).all())
    del flip
    assert bool((keys[vo.long()] == ko).all())
    assert bool(((ko[1:] != ko[:-1]) | (vo[1:] > vo[:-1])).all())


@pytest.mark.parametrize("n", [1000, (1 << 20) + 3])
def test_in_place(n):
    _check(inputs.keyset("d", n, seed=3).keys, inplace=True)


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_every_tile_shape(shape):
    from paper_cs_0004013_amd import binding
    binding.ap_set_pass_shape(shape)
    try:
        _check(inputs.keyset("a", 300_007, seed=shape).keys)
    finally:
        binding.ap_set_pass_shape(-1)


def test_mask_rank_path():
    from paper_cs_0004013_amd import binding
    binding.ap_set_rank_mode(1)
    try:
        _check(inputs.keyset("e", (1 << 22) + 5, seed=2).keys)
    finally:
        binding.ap_set_rank_mode(0)


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_mask_rank_every_tile_shape(shape):
    """The mask rank on every pairs tile (its 16K tile is 8 waves x 32 keys, not the atomic rank's
    16 x 16), with a ragged last tile and runs of equal keys."""
    from paper_cs_0004013_amd import binding
    binding.ap_set_rank_mode(1)
    binding.ap_set_pass_shape(shape)
    try:
        _check(inputs.keyset("d", 200_003 + shape, seed=40 + shape).keys)
    finally:
        binding.ap_set_pass_shape(-1)
        binding.ap_set_rank_mode(0)


def test_argsort_helper():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    keys = inputs.keyset("c", 100_000, seed=1).keys ^ (np.arange(100_000, dtype=np.uint32) % 7)
    t, _ = to_dev(keys)
    k_out, perm = binding.argsort_u32(t)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(perm), np.argsort(keys, kind="stable").astype(np.uint32))
    assert np.array_equal(to_host(k_out), np.sort(keys))


def test_invalid_arguments():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    a = torch.zeros(1000, dtype=torch.int32, device="cuda")
    b = torch.zeros(1000, dtype=torch.int32, device="cuda")
    c = torch.zeros(1000, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.ApError):
        binding.ap_sort_pairs_u32(a, b, a, c)      # keys in place, values not
    with pytest.raises(binding.ApError):
        binding.ap_sort_pairs_u32(a, b, c, a)      # value output overlaps the key input
    big = torch.zeros(2000, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.ApError):
        binding.ap_sort_pairs_u32(big[:1000], big[500:1500], c, b)  # key and value inputs overlap


def test_workspace_variant():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    keys = inputs.keyset("b", 500_001, seed=9).keys
    vals = np.arange(keys.size, dtype=np.uint32)[::-1].copy()
    ws = torch.empty(binding.ap_sort_pairs_workspace_bytes(keys.size), dtype=torch.uint8, device="cuda")
    binding.ap_workspace_init(ws)
    k_in, _ = to_dev(keys)
    v_in, _ = to_dev(vals)
    k_out = torch.empty_like(k_in)
    v_out = torch.empty_like(v_in)
    spl = torch.empty(63, dtype=torch.int32, device="cuda")
    for _ in range(2):
        binding.ap_sort_pairs_u32_ws(k_in, v_in, k_out, v_out, 64, spl, ws)
        torch.cuda.synchronize()
        wk, wv = oracle.sort_pairs_u32(keys, vals)
        assert np.array_equal(to_host(k_out), wk) and np.array_equal(to_host(v_out), wv)
        assert np.array_equal(to_host(spl), oracle.splitters(wk, 64))
