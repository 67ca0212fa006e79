"""Parity of the single-array sort (A1-A7) with the CPU oracle, through the C ABI.

Every result is compared element by element with the oracle (bit-exact: integer work), and the
splitters with the oracle's; the invariant checks of tests/invariants.py run as well.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_cs_0004013_amd import inputs
from tests import invariants as inv
from tests.gpu_util import announce, gpu_sort, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _check(keys: np.ndarray, P: int = 64, **kw):
    announce(f"sort n={keys.size} P={P} {kw}")
    out, spl = gpu_sort(keys, P, **kw)
    want = oracle.sort_u32(keys)
    assert out.size == want.size
    bad = np.flatnonzero(out != want)
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    assert np.array_equal(spl, oracle.splitters(want, P))
    return out, spl


def test_uniform_2pow20_config():
    """2^20 i.i.d. uniform keys in [0, 2^31-1], seed 0, P = 64."""
    ks = inputs.keyset("a", 1 << 20, seed=0)
    out, spl = _check(ks.keys)
    assert inv.is_nondecreasing(out) and inv.same_multiset(out, ks.keys)
    inv.check_splitters(out, 64, spl)


# around the tile-shape thresholds by size (2^17, 2^20, 2^22) and the one-launch limit (16384)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 63, 64, 65, 255, 256, 257, 2047, 2048, 2049, 8191, 8192,
                               8193, 16384, 16385, 100_000, (1 << 17) - 1, 1 << 17, (1 << 20) - 1, 1 << 20,
                               (1 << 20) + 7, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, 3 * 8192 * 7 + 5])
def test_sizes_full_range(n):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)  # bit 31 set too
    _check(keys)


# from 2^23 keys on, the keys-only passes before the last store plainly and the last pass with the
# non-temporal hint; below, every pass uses the hint: both sides of the boundary and a large ragged
# size, with the atomic rank (32K tile) and the mask rank (16K)
@pytest.mark.parametrize("rank_mode", [0, 1])
@pytest.mark.parametrize("n", [(1 << 23) - 1, 1 << 23, (1 << 26) + 3])
def test_store_hint_boundaries(n, rank_mode):
    from paper_cs_0004013_amd import binding
    rng = np.random.default_rng(n + rank_mode)
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    binding.ap_set_rank_mode(rank_mode)
    try:
        _check(keys)
    finally:
        binding.ap_set_rank_mode(0)


@pytest.mark.parametrize("dist", inputs.DISTS)
def test_distributions_2pow22(dist):
    _check(inputs.keyset(dist, (1 << 22) + 13, seed=11).keys)


@pytest.mark.parametrize("seed", range(1, 6))
@pytest.mark.parametrize("dist", inputs.DISTS)
def test_distributions_full_size(seed, dist):
    """2^26 keys, every (seed 1-5) x (distribution (a)-(e)) pair; the benchmark times the
    diagonal (seed i with distribution i)."""
    _check(inputs.keyset(dist, 1 << 26, seed=seed).keys)


def test_adversarial_full_size():
    """2^27 keys: top 16 bits take 4 values, hot keys duplicated 1000x."""
    _check(inputs.adversarial(1 << 27, seed=0).keys)


@pytest.mark.parametrize("n", [0, 1, 5, 64, 1000, 8193, 1 << 20])
@pytest.mark.parametrize("P", [1, 2, 3, 63, 64, 65])
def test_cells_and_splitters(n, P):
    rng = np.random.default_rng(n + P)
    keys = rng.integers(0, 1 << 31, size=n, dtype=np.uint64).astype(np.uint32)
    _check(keys, P)
    if n:
        _check(keys, n + 1)       # more cells than keys: empty cells get all-ones splitters


@pytest.mark.parametrize("n", [1000, 65_537, (1 << 22) + 3])
def test_in_place(n):
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    _check(keys, inplace=True)
    _check(keys >> np.uint32(8), inplace=True)   # 3 passes run: odd count in place needs a copy
    _check(np.full(n, 77, np.uint32), inplace=True)


@pytest.mark.parametrize("pad", [1, 2, 3])
def test_unaligned_start(pad):
    keys = inputs.keyset("d", (1 << 20) + 3, seed=pad).keys
    _check(keys, pad_front=pad)


def test_closed_forms():
    rng = np.random.default_rng(0)
    n = (1 << 20) + 123
    perm = rng.permutation(n).astype(np.uint32)
    out, spl = _check(perm)
    assert np.array_equal(out, np.arange(n, dtype=np.uint32))
    asc = np.sort(rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32))
    _check(asc)
    _check(asc[::-1].copy())


def _plan(keys: np.ndarray, bits: int):
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    D = (32 + bits - 1) // bits
    t_in, _ = to_dev(keys)
    h = torch.zeros(D << bits, dtype=torch.int32, device="cuda")
    p = torch.zeros(D + 1, dtype=torch.int32, device="cuda")
    binding.ap_digit_plan_u32(t_in, bits, h, p)
    torch.cuda.synchronize()
    return to_host(h).reshape(D, 1 << bits), to_host(p)


@pytest.mark.parametrize("bits", [4, 5, 6, 7, 8, 9, 10, 11])
@pytest.mark.parametrize("dist", ["a", "c", "e"])
def test_digit_histograms_and_plan(bits, dist):
    """A1/A2: bucket counts of every digit equal the oracle's; a pass runs iff its digit column
    is not constant."""
    keys = inputs.keyset(dist, 300_001, seed=bits).keys
    announce(f"digit plan bits={bits} dist={dist}")
    h, plan = _plan(keys, bits)
    D = h.shape[0]
    run = []
    for d in range(D):
        want = oracle.digit_hist(keys, d * bits, min(bits, 32 - d * bits))
        got = h[d, :want.size].astype(np.uint64)
        assert np.array_equal(got, want), f"digit {d}"
        assert not h[d, want.size:].any()
        run.append(0 if want.max() == keys.size else 1)
    assert plan[:D].tolist() == run
    assert plan[D] == sum(run)


def test_maximum_size_counts_and_sort():
    """n = 2^30 - 1, the largest n accepted.  The histogram's workgroups each count up to 4092
    keys per thread into 16-bit per-lane counters; with constant keys one counter of every copy
    takes all of them, its worst case.  Then two sorts at that size: a two-valued input checked
    on the device by counts, and a uniform full-range input compared element by element with the
    oracle on the host."""
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    n = (1 << 30) - 1
    announce(f"maximum size n={n}: constant-key histogram")
    t = torch.full((n,), 0x12345678, dtype=torch.int32, device="cuda")
    h = torch.zeros(4 * 256, dtype=torch.int32, device="cuda")
    p = torch.zeros(5, dtype=torch.int32, device="cuda")
    binding.ap_digit_plan_u32(t, 8, h, p)
    hh = to_host(h).reshape(4, 256)
    for d in range(4):
        want = np.zeros(256, np.uint32)
        want[(0x12345678 >> (8 * d)) & 255] = n
        assert np.array_equal(hh[d], want), f"digit {d}"
    assert to_host(p).tolist() == [0, 0, 0, 0, 0]
    del t

    announce(f"maximum size n={n}: two-valued sort")
    g = torch.Generator(device="cuda").manual_seed(5)
    keys = torch.randint(0, 2, (n,), device="cuda", generator=g, dtype=torch.int32)
    keys.mul_(-8).add_(7)            # 7 or -1 (= 0xFFFFFFFF unsigned)
    c7 = int((keys == 7).sum())
    out = torch.empty_like(keys)
    spl = torch.empty(63, dtype=torch.int32, device="cuda")
    binding.ap_sort_u32(keys, out, 64, spl)
    torch.cuda.synchronize()
    assert bool((out[:c7] == 7).all()) and bool((out[c7:] == -1).all())

    announce(f"maximum size n={n}: uniform sort, element-wise against the oracle")
    keys = torch.randint(-(1 << 31), 1 << 31, (n,), device="cuda", generator=g, dtype=torch.int32)
    binding.ap_sort_u32(keys, out, 64, spl)
    torch.cuda.synchronize()
    h_keys = to_host(keys)
    del keys
    got = to_host(out)
    want = oracle.sort_u32(h_keys)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    assert np.array_equal(to_host(spl), oracle.splitters(want, 64))


def test_pass_skip_counts():
    keys24 = inputs.keyset("a", 100_000, 3).keys >> np.uint32(7)      # < 2^24: 3 passes
    assert _plan(keys24, 8)[1][4] == 3
    assert _plan(np.full(1000, 9, np.uint32), 8)[1][4] == 0            # constant: 0 passes
    adv = inputs.adversarial(1 << 20, 0).keys                           # 4 top values: 4 passes
    assert _plan(adv, 8)[1][4] == 4


def test_repeatable_bitwise():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    for keys in (inputs.keyset("a", (1 << 22) + 5, 1).keys, inputs.keyset("e", 1 << 22, 2).keys):
        announce(f"repeat n={keys.size}")
        t_in, _ = to_dev(keys)
        t_out = torch.empty_like(t_in)
        first = None
        for _ in range(20):
            binding.ap_sort_u32(t_in, t_out, 64, None)
            cur = t_out.clone()
            if first is None:
                first = cur
            else:
                assert torch.equal(cur, first)
        assert np.array_equal(to_host(first), oracle.sort_u32(keys))


def test_caller_workspace():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    n = (1 << 21) + 9
    keys = inputs.keyset("d", n, 4).keys
    ws = torch.empty(binding.ap_sort_workspace_bytes(n) + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + binding.ap_sort_workspace_bytes(n)]
    binding.ap_workspace_init(ws)
    t_in, _ = to_dev(keys)
    t_out = torch.empty_like(t_in)
    spl = torch.empty(63, dtype=torch.int32, device="cuda")
    for _ in range(3):
        binding.ap_sort_u32_ws(t_in, t_out, 64, spl, ws)
    torch.cuda.synchronize()
    want = oracle.sort_u32(keys)
    assert np.array_equal(to_host(t_out), want)
    assert np.array_equal(to_host(spl), oracle.splitters(want, 64))
    small = keys[:1000].copy()                         # smaller call on the same workspace
    t2, _ = to_dev(small)
    o2 = torch.empty_like(t2)
    binding.ap_sort_u32_ws(t2, o2, 64, spl, ws)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(o2), oracle.sort_u32(small))


def test_invalid_args_raise():
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    base = torch.zeros(101, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.ApError):
        binding.ap_sort_u32(base[0:100], base[1:101], 64)      # partial overlap
    with pytest.raises(binding.ApError):
        binding.ap_sort_u32(base[0:100], base[0:100], 0)       # P < 1


def test_rank_self_check_passed():
    """The device check of the LDS lane-order property ran and passed, so the atomic rank is used."""
    from paper_cs_0004013_amd import binding
    _check(inputs.keyset("a", 5000, 1).keys)
    assert binding.ap_rank_check_state() == 1


@pytest.mark.parametrize("dist", ["a", "d", "e"])
@pytest.mark.parametrize("n", [12_345, 70_001, (1 << 19) + 3, (1 << 21) + 9, (1 << 22) + 77])
def test_match_rank_path(dist, n):
    """The order-agnostic mask rank gives the same (oracle) result: the one-launch path, and every
    device-wide tile shape by size (4K, 8K and 16K keys; the 16K tile where 32K would be used)."""
    from paper_cs_0004013_amd import binding
    binding.ap_set_rank_mode(1)
    try:
        _check(inputs.keyset(dist, n, 21).keys)
    finally:
        binding.ap_set_rank_mode(0)



@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [70_001, (1 << 20) + 77])
def test_pass_shapes(shape, n):
    """Every tile shape gives the oracle's result at sizes with a ragged last tile (by size, the
    32K-key tile runs only from 2^22 keys on and the 4K-key tile only below 2^17)."""
    from paper_cs_0004013_amd import binding
    binding.ap_set_pass_shape(shape)
    try:
        _check(inputs.keyset("e" if n & 1 else "a", n, 31).keys)
    finally:
        binding.ap_set_pass_shape(-1)


def test_workspace_sort_graph_capture_replay():
    """ap_sort_u32_ws allocates nothing and never synchronises, so it can be captured in a HIP
    graph; every replay (with eager work and synchronisation in between) must give the oracle's
    result for the input then in the buffer."""
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    n = (1 << 20) + 333
    announce(f"graph capture of the workspace sort n={n}")
    ws = torch.empty(binding.ap_sort_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    binding.ap_workspace_init(ws)
    t_in = torch.zeros(n, dtype=torch.int32, device="cuda")
    t_out = torch.empty_like(t_in)
    spl = torch.empty(63, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        binding.ap_sort_u32_ws(t_in, t_out, 64, spl, ws, stream=s)
    for rep, dist in enumerate(["a", "e", "c", "d", "a"]):
        keys = inputs.keyset(dist, n, 40 + rep).keys
        t_in.copy_(to_dev(keys)[0])        # eager work between replays
        t_out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want = oracle.sort_u32(keys)
        assert np.array_equal(to_host(t_out), want), f"replay {rep}"
        assert np.array_equal(to_host(spl), oracle.splitters(want, 64)), f"replay {rep} splitters"


@pytest.mark.parametrize("rank_mode", [0, 1])
def test_small_arrays_one_launch(rank_mode):
    """Arrays of at most 16384 keys take the one-workgroup path of ap_sort_u32; the same keys
    through ap_sort_u32_ws take the device-wide passes: both equal the oracle, at every tile edge
    of the small path, in place, and with more cells than keys."""
    torch = torch_cuda()
    from paper_cs_0004013_amd import binding
    binding.ap_set_rank_mode(rank_mode)
    try:
        rng = np.random.default_rng(77)
        ws = torch.empty(binding.ap_sort_workspace_bytes(16384), dtype=torch.uint8, device="cuda")
        binding.ap_workspace_init(ws)
        for n in (1, 2, 3, 100, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 16383, 16384):
            for dist in ("full", "e", "c"):
                if dist == "full":
                    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
                else:
                    keys = inputs.keyset(dist, n, seed=n).keys
                announce(f"small n={n} dist={dist} rank_mode={rank_mode}")
                want = oracle.sort_u32(keys)
                for P in (64, n + 1):
                    out, spl = gpu_sort(keys, P)
                    assert np.array_equal(out, want) and np.array_equal(spl, oracle.splitters(want, P)), (n, P)
                out, _ = gpu_sort(keys, 5, inplace=True)
                assert np.array_equal(out, want)
                t_in, _ = to_dev(keys)
                t_out = torch.empty_like(t_in)
                binding.ap_sort_u32_ws(t_in, t_out, 1, None, ws)
                torch.cuda.synchronize()
                assert np.array_equal(to_host(t_out), want)
    finally:
        binding.ap_set_rank_mode(0)
