"""Parity of the batched segmented sort (A8) with the CPU oracle, through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_cs_0004013_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _run(keys: np.ndarray, offsets: np.ndarray, cfg: int | None = None, pad_front: int = 0):
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    t_keys, _ = to_dev(keys, pad_front)
    t_off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint32).view(np.int32)).to("cuda")
    t_st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    saved = binding.segmented_groups()
    if cfg is not None:
        binding.ap_segmented_set_config(cfg)
    try:
        binding.ap_sort_u32_segmented(t_keys, t_off, t_st)
        torch.cuda.synchronize()
    finally:
        binding.set_segmented_groups(saved)
    return to_host(t_keys), int(to_host(t_st)[0])


def _check(keys, offsets, **kw):
    announce(f"segmented nseg={len(offsets) - 1} n={keys.size} {kw}")
    got, status = _run(keys, offsets, **kw)
    want = oracle.sort_segmented(keys, offsets.astype(np.uint64))
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    assert status == 0
    return got


def _batch(lengths, seed=0):
    L = np.asarray(lengths, dtype=np.int64)
    keys, off, _ = inputs.segment_keys(L)
    return keys, off


def test_log_uniform_batch_512():
    """512 segments, lengths log-uniform in [64, 2^18], distributions (a)-(e) by segment seed."""
    L = inputs.segment_lengths(512, seed=0)
    keys, off = _batch(L)
    _check(keys, off)


def test_group_split_table():
    """A custom four-group table (different configurations per length range) gives oracle results."""
    from paper_cs_0004013_amd import binding
    saved = binding.segmented_groups()
    try:
        binding.set_segmented_groups([(15, 31, 1), (12, 14, 5), (9, 11, 2), (1, 8, 4)])
        L = inputs.segment_lengths(200, seed=8, lo=2, hi=1 << 17)
        keys, off = _batch(L)
        _check(keys, off)
    finally:
        binding.set_segmented_groups(saved)


N_CONFIGS = 12  # compiled-in configurations (digit widths 4, 6, 8, 10, 11)


def test_config_count():
    from paper_cs_0004013_amd import binding
    assert binding.ap_segmented_num_configs() == N_CONFIGS
    assert sorted({binding.ap_segmented_config_info(c)[0] for c in range(N_CONFIGS)}) == [4, 6, 8, 10, 11]


@pytest.mark.parametrize("cfg", range(N_CONFIGS))
def test_every_config(cfg):
    L = inputs.segment_lengths(96, seed=cfg + 1, lo=2, hi=1 << 16)
    L[::7] = 0
    L[::11] = 1
    keys, off = _batch(L)
    _check(keys, off, cfg=cfg)


def test_boundary_lengths():
    """Lengths at every tile-size boundary +-1 and a few multi-tile sizes."""
    Ls = []
    for T in (1024, 2048, 4096, 8192, 16384):
        Ls += [T - 1, T, T + 1]
    Ls += [0, 1, 2, 3, 63, 64, 65, 3 * 8192 + 5, 100_000, 1 << 18]
    keys, off = _batch(Ls)
    _check(keys, off)


def test_single_large_segment():
    keys, off = _batch([(1 << 20) + 3])
    _check(keys, off)


def test_constant_and_clustered_segments():
    rng = np.random.default_rng(3)
    parts, L = [], []
    for i, n in enumerate([70_000, 5000, 40_000, 9000]):
        if i % 2 == 0:
            parts.append(np.full(n, 123456 + i, np.uint32))
        else:
            parts.append((rng.integers(0, 4, n).astype(np.uint32) << np.uint32(24)) | np.uint32(77))
        L.append(n)
    keys = np.concatenate(parts)
    off = np.zeros(len(L) + 1, np.int64)
    np.cumsum(L, out=off[1:])
    _check(keys, off.astype(np.uint32))


@pytest.mark.parametrize("cfg", [None, 0, 3, 10])
def test_segments_of_equal_key_runs(cfg):
    """Segments made of runs of equal keys (lengths 1..199): rank slots switch between
    all-lanes-equal digits and mixed ones, in every configuration's digit sweeps."""
    rng = np.random.default_rng(99)
    lens = rng.integers(1, 200, size=8000)
    vals = rng.integers(0, 1 << 32, size=lens.size, dtype=np.uint64).astype(np.uint32)
    keys = np.repeat(vals, lens)
    seg = np.concatenate([[0], np.sort(rng.choice(np.arange(1, keys.size), size=63, replace=False)), [keys.size]])
    _check(keys, seg.astype(np.uint32), cfg=cfg)


def test_maximum_total_size():
    """n_total = 2^30 - 1 full-range keys in 4096 segments of random lengths, compared element by
    element with the oracle's per-segment sort on the host."""
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    n = (1 << 30) - 1
    rng = np.random.default_rng(4)
    cuts = np.sort(rng.choice(np.arange(1, n), size=4095, replace=False))
    off = np.concatenate([[0], cuts, [n]]).astype(np.uint32)
    announce(f"segmented maximum total n={n}")
    g = torch.Generator(device="cuda").manual_seed(4)
    keys = torch.randint(-(1 << 31), 1 << 31, (n,), device="cuda", generator=g, dtype=torch.int32)
    h_keys = to_host(keys)
    t_off = torch.from_numpy(off.view(np.int32)).to("cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    binding.ap_sort_u32_segmented(keys, t_off, st)
    torch.cuda.synchronize()
    assert int(st[0]) == 0
    got = to_host(keys)
    del keys
    want = oracle.sort_segmented(h_keys, off.astype(np.uint64))
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"


def test_benchmark_batch_4096():
    """The benchmark's batch itself: 4096 segments, lengths log-uniform in [64, 2^18] (seed 0),
    segment s drawn with seed s, against the oracle element by element."""
    L = inputs.segment_lengths(4096, seed=0)
    keys, off = _batch(L)
    _check(keys, off)


@pytest.fixture
def order_agnostic_rank():
    """Rank mode 1: the segmented kernels rank with ballots instead of lane-ordered LDS atomics."""
    from paper_cs_0004013_amd import binding
    binding.ap_set_rank_mode(1)
    try:
        yield
    finally:
        binding.ap_set_rank_mode(0)


def test_ballot_rank_log_uniform_512(order_agnostic_rank):
    L = inputs.segment_lengths(512, seed=0)
    keys, off = _batch(L)
    _check(keys, off)


@pytest.mark.parametrize("cfg", range(N_CONFIGS))
def test_ballot_rank_every_config(cfg, order_agnostic_rank):
    L = inputs.segment_lengths(64, seed=cfg + 40, lo=2, hi=1 << 16)
    L[::9] = 1
    keys, off = _batch(L)
    _check(keys, off, cfg=cfg)


@pytest.mark.parametrize("cfg", [None, 3, 10])
def test_ballot_rank_equal_key_runs(cfg, order_agnostic_rank):
    rng = np.random.default_rng(98)
    lens = rng.integers(1, 200, size=6000)
    vals = rng.integers(0, 1 << 32, size=lens.size, dtype=np.uint64).astype(np.uint32)
    keys = np.repeat(vals, lens)
    seg = np.concatenate([[0], np.sort(rng.choice(np.arange(1, keys.size), size=47, replace=False)), [keys.size]])
    _check(keys, seg.astype(np.uint32), cfg=cfg)


def test_ballot_rank_graph_recaptured():
    """Switching the rank mode between calls with identical arguments re-captures the graph: the
    replayed sequence never keeps the other rank's kernels."""
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    L = inputs.segment_lengths(48, seed=12)
    keys, off = _batch(L)
    want = oracle.sort_segmented(keys, off.astype(np.uint64))
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            t_off = torch.from_numpy(off.view(np.int32)).to("cuda")
            t_keys, _ = to_dev(keys)
            for mode in (0, 1, 1, 0):
                binding.ap_set_rank_mode(mode)
                t_keys.copy_(torch.from_numpy(keys.view(np.int32)).to("cuda"))
                binding.ap_sort_u32_segmented(t_keys, t_off)
                s.synchronize()
                assert np.array_equal(to_host(t_keys), want), mode
    finally:
        binding.ap_set_rank_mode(0)


def test_full_range_keys_and_unaligned_segments():
    rng = np.random.default_rng(9)
    keys = rng.integers(0, 1 << 32, size=300_001, dtype=np.uint64).astype(np.uint32)
    cuts = np.sort(rng.choice(np.arange(1, keys.size), size=40, replace=False))
    off = np.concatenate([[3], cuts, [keys.size - 2]]).astype(np.uint32)   # keys outside stay put
    got = _check(keys, off, pad_front=1)
    assert np.array_equal(got[:3], keys[:3]) and np.array_equal(got[-2:], keys[-2:])


def test_invalid_offsets_reported():
    keys, off = _batch([1000, 2000, 3000])
    bad = off.copy()
    bad[2] = bad[1] - 10                 # segment 1 decreasing
    got, status = _run(keys, bad)
    assert status == 1                   # AP_ERR_INVALID
    assert np.array_equal(got, keys)     # nothing sorted
    beyond = off.copy()
    beyond[-1] = keys.size + 1           # past n_total
    got, status = _run(keys, beyond)
    assert status == 1 and np.array_equal(got, keys)
    got, status = _run(keys, off)        # valid again afterwards (control block was reset)
    assert status == 0 and np.array_equal(got, oracle.sort_segmented(keys, off.astype(np.uint64)))


def test_graph_replay_and_recapture():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    L = inputs.segment_lengths(64, seed=5)
    keys, off = _batch(L)
    want = oracle.sort_segmented(keys, off.astype(np.uint64))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t_off = torch.from_numpy(off.view(np.int32)).to("cuda")
        t_keys, _ = to_dev(keys)
        for rep in range(4):             # first call captures, the rest replay
            t_keys.copy_(torch.from_numpy(keys.view(np.int32)).to("cuda"))
            binding.ap_sort_u32_segmented(t_keys, t_off)
            s.synchronize()
            assert np.array_equal(to_host(t_keys), want), rep
        keys2, off2 = _batch(inputs.segment_lengths(33, seed=6))
        t2, _ = to_dev(keys2)
        t_off2 = torch.from_numpy(off2.view(np.int32)).to("cuda")
        binding.ap_sort_u32_segmented(t2, t_off2)
        s.synchronize()
        assert np.array_equal(to_host(t2), oracle.sort_segmented(keys2, off2.astype(np.uint64)))


def test_empty_batch():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    t = torch.zeros(4, dtype=torch.int32, device="cuda")
    binding.ap_sort_u32_segmented(t, torch.zeros(1, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()


@pytest.fixture
def long_min():
    """Sets the long-segment threshold for one test and restores it."""
    from paper_cs_0004013_amd import binding
    saved = binding.ap_segmented_get_long_min()
    yield binding.ap_segmented_set_long_min
    binding.ap_segmented_set_long_min(saved)


@pytest.mark.parametrize("rank_mode", [0, 1])
def test_long_segments_device_wide(long_min, rank_mode):
    """A low threshold sends most segments through the device-wide passes: lengths at flat-tile
    boundaries (16K and 32K keys +-1), constant segments (no pass runs), keys below 2^24 (three
    passes: the copy back), full-range keys, next to short segments sorted by one workgroup."""
    from paper_cs_0004013_amd import binding
    long_min(5000)
    rng = np.random.default_rng(21)
    parts, L = [], []
    lens = [16383, 16384, 16385, 32767, 32768, 32769, 5000, 4999, 100_003, 3 * 32768 + 7, 70_000, 9000, 12,
            250_000, 65_536]
    for i, n in enumerate(lens):
        kind = i % 4
        if kind == 0:
            k = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
        elif kind == 1:
            k = np.full(n, 0xDEADBEEF - i, np.uint32)
        elif kind == 2:
            k = rng.integers(0, 1 << 24, size=n, dtype=np.uint64).astype(np.uint32)
        else:
            k = inputs.dist_keys("e", n, rng)
        parts.append(k)
        L.append(n)
    keys = np.concatenate(parts)
    off = np.zeros(len(L) + 1, np.int64)
    np.cumsum(L, out=off[1:])
    binding.ap_set_rank_mode(rank_mode)
    try:
        _check(keys, off.astype(np.uint32))
        _check(keys, off.astype(np.uint32))          # graph replay / second call reuses the plans
    finally:
        binding.ap_set_rank_mode(0)


def test_long_segments_mixed_batch(long_min):
    """4 segments of 2^24 keys (distributions a, c, d, e) and 4092 log-uniform short segments,
    with the default threshold (2^20): the long ones go device-wide."""
    long_min(1 << 20)
    rng = np.random.default_rng(5)
    short = inputs.segment_lengths(4092, seed=3, lo=64, hi=1 << 14)
    L = np.concatenate([[1 << 24] * 4, short]).astype(np.int64)
    L = L[rng.permutation(L.size)]
    keys, off = _batch(L)
    _check(keys, off)


def test_single_segment_2pow28():
    """One segment of 2^28 keys (dist d) in a buffer with a few keys before and after it."""
    n = 1 << 28
    keys = inputs.keyset("d", n + 10, seed=8).keys
    off = np.array([3, n + 3], dtype=np.uint32)
    got = _check(keys, off)
    assert np.array_equal(got[:3], keys[:3]) and np.array_equal(got[-7:], keys[-7:])
