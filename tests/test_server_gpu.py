"""Served form (A9): requests submitted to the ap_server_* request loop are sorted exactly like the
oracle, alone and inside a mix; admission, fault isolation and cancellation behave as specified."""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
from paper_cs_0004013_amd import inputs
from tests.gpu_util import announce, to_host, torch_cuda

pytestmark = pytest.mark.gpu

AP_OK, AP_ERR_BUDGET, AP_ERR_TIMEOUT, AP_ERR_DEVICE, AP_ERR_CANCELLED = 0, 4, 6, 7, 8


class Pool:
    """Five device-resident key pools (one per distribution); requests are windows into them."""

    def __init__(self, keys_per_pool: int):
        torch = torch_cuda()
        self.host = {d: inputs.keyset(d, keys_per_pool, seed=100 + i).keys for i, d in enumerate(inputs.DISTS)}
        self.dev = {d: torch.from_numpy(k.view(np.int32)).to("cuda") for d, k in self.host.items()}
        self.size = keys_per_pool


def _requests(pool: Pool, nreq: int, lo: int, hi: int, seed: int = 0):
    tr = inputs.request_trace(nreq, rate_per_s=1e6, pool_keys=pool.size, seed=seed, lo=lo, hi=hi)
    return tr


def _run(server, pool, reqs, P=64, gap_s=0.0):
    torch = torch_cuda()
    outs, spls, tickets = [], [], []
    for r in reqs:
        src = pool.dev[r.dist][r.pool_offset:r.pool_offset + r.n]
        out = torch.empty(r.n, dtype=torch.int32, device="cuda")
        spl = torch.empty(P - 1, dtype=torch.int32, device="cuda")
        outs.append(out)
        spls.append(spl)
        tickets.append(server.submit(src, out, P, spl))
        if gap_s:
            time.sleep(gap_s)
    statuses = [server.wait(t) for t in tickets]
    torch.cuda.synchronize()
    return statuses, [to_host(o) for o in outs], [to_host(s) for s in spls]


def _want(pool, r, P=64):
    w = oracle.sort_u32(pool.host[r.dist][r.pool_offset:r.pool_offset + r.n])
    return w, oracle.splitters(w, P)


def test_mixed_sizes_match_oracle():
    from paper_cs_0004013_amd import binding
    pool = Pool(1 << 21)
    reqs = _requests(pool, 160, 1 << 4, 1 << 20, seed=1)
    announce("server mixed 160 requests")
    with binding.Server(hbm_budget_bytes=1 << 30, num_streams=4, max_batch=64, alone_min_keys=1 << 18) as srv:
        st, outs, spls = _run(srv, pool, reqs)
        stats = srv.stats()
    assert all(s == AP_OK for s in st)
    for r, o, sp in zip(reqs, outs, spls):
        w, ws = _want(pool, r)
        assert np.array_equal(o, w) and np.array_equal(sp, ws), r
    assert stats["completed"] == len(reqs)
    assert stats["batches"] < len(reqs)          # short requests were batched
    assert stats["alone"] >= 1                   # long ones ran device-wide


@pytest.mark.parametrize("rank_mode", [0, 1])
def test_alone_vs_mix_identical(rank_mode):
    """Each request gives byte-identical output run alone and inside a Poisson mix, with the
    default rank and with the order-agnostic one (rank mode 1)."""
    from paper_cs_0004013_amd import binding
    pool = Pool(1 << 20)
    reqs = _requests(pool, 48, 1 << 10, 1 << 19, seed=2)
    announce(f"server alone vs mix, rank mode {rank_mode}")
    binding.ap_set_rank_mode(rank_mode)
    try:
        _alone_vs_mix(binding, pool, reqs)
    finally:
        binding.ap_set_rank_mode(0)


def _alone_vs_mix(binding, pool, reqs):
    with binding.Server(hbm_budget_bytes=1 << 29, num_streams=3, max_batch=32, alone_min_keys=1 << 18) as srv:
        alone = []
        for r in reqs:                            # one at a time: each runs alone
            st, o, sp = _run(srv, pool, [r])
            assert st == [AP_OK]
            alone.append((o[0], sp[0]))
        rng = np.random.default_rng(0)
        order = rng.permutation(len(reqs))
        torch = torch_cuda()
        outs, spls, tks = {}, {}, {}
        for i in order:                           # the mix: exponential gaps, arrivals during runs
            r = reqs[i]
            src = pool.dev[r.dist][r.pool_offset:r.pool_offset + r.n]
            outs[i] = torch.empty(r.n, dtype=torch.int32, device="cuda")
            spls[i] = torch.empty(63, dtype=torch.int32, device="cuda")
            tks[i] = srv.submit(src, outs[i], 64, spls[i])
            time.sleep(float(rng.exponential(20e-6)))
        assert all(srv.wait(tks[i]) == AP_OK for i in order)
        torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        w, ws = _want(pool, r)
        assert np.array_equal(to_host(outs[i]), alone[i][0]) and np.array_equal(alone[i][0], w)
        assert np.array_equal(to_host(spls[i]), alone[i][1]) and np.array_equal(alone[i][1], ws)


def test_admission_under_tiny_budget():
    from paper_cs_0004013_amd import binding
    torch = torch_cuda()
    pool = Pool(1 << 20)
    with binding.Server(hbm_budget_bytes=8 << 20, num_streams=2, max_batch=16, alone_min_keys=1 << 30) as srv:
        n_over = (1 << 21) + 64                      # 8 MiB + 256 B of scratch: more than the whole budget
        big = torch.empty(n_over, dtype=torch.int32, device="cuda")
        out = torch.empty_like(big)
        st, _ = srv.try_submit_ptr(big.data_ptr(), out.data_ptr(), n_over, 1)
        assert st == AP_ERR_BUDGET
        # one request whose 4 MiB of scratch is half the budget (more than an even share of two slots)
        # runs; then 40 that each fit and together exceed the budget
        reqs = [inputs.Request(-1, 1 << 20, "a", 0, 0.0)] + _requests(pool, 40, 1 << 16, 1 << 19, seed=3)
        st, outs, spls = _run(srv, pool, reqs)
        assert all(s == AP_OK for s in st)
        for r, o, sp in zip(reqs, outs, spls):
            w, ws = _want(pool, r)
            assert np.array_equal(o, w) and np.array_equal(sp, ws)
        stats = srv.stats()
        assert stats["scratch_budget_bytes"] == 8 << 20
        assert (4 << 20) <= stats["scratch_peak_bytes"] <= (8 << 20)
        assert 0 <= stats["queue_p50_us"] <= stats["p50_us"]


def test_injected_fault_fails_only_its_ticket():
    from paper_cs_0004013_amd import binding
    torch = torch_cuda()
    pool = Pool(1 << 18)
    with binding.Server(hbm_budget_bytes=1 << 28, num_streams=2) as srv:
        tk, outs = [], []
        for i in range(12):
            src = pool.dev["d"][i * 1000:(i + 1) * 1000]
            out = torch.empty(1000, dtype=torch.int32, device="cuda")
            outs.append(out)
            tk.append(srv.submit_ptr(src.data_ptr(), out.data_ptr(), 1000, 1, None,
                                     binding.AP_SUBMIT_INJECT_FAULT if i == 5 else 0))
        st = [srv.wait(t) for t in tk]
        torch.cuda.synchronize()
    assert st[5] == AP_ERR_DEVICE and all(s == AP_OK for i, s in enumerate(st) if i != 5)
    for i in range(12):
        if i != 5:
            assert np.array_equal(to_host(outs[i]), oracle.sort_u32(pool.host["d"][i * 1000:(i + 1) * 1000]))


def test_edge_requests_in_place_empty_tiny():
    from paper_cs_0004013_amd import binding
    torch = torch_cuda()
    with binding.Server(hbm_budget_bytes=1 << 28, num_streams=2, alone_min_keys=1 << 16) as srv:
        rng = np.random.default_rng(4)
        cases = []
        for n in (0, 1, 2, 5, 8191, 8192, 8193, 70_000, (1 << 16) + 3):
            keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
            t = torch.from_numpy(keys.view(np.int32)).to("cuda") if n else torch.empty(0, dtype=torch.int32,
                                                                                       device="cuda")
            spl = torch.empty(99, dtype=torch.int32, device="cuda")
            tk = srv.submit_ptr(t.data_ptr() if n else 0, t.data_ptr() if n else 0, n, 100, spl.data_ptr())
            cases.append((keys, t, spl, tk))
        for keys, t, spl, tk in cases:
            assert srv.wait(tk) == AP_OK
        torch.cuda.synchronize()
        for keys, t, spl, tk in cases:
            w = oracle.sort_u32(keys)
            assert np.array_equal(to_host(t) if keys.size else keys, w)
            assert np.array_equal(to_host(spl), oracle.splitters(w, 100))


def test_lone_short_requests_one_launch():
    """Requests submitted one at a time form batches of one; those of at most 16,384 keys take the
    one-launch single-array sort, longer ones the segmented kernel.  Both match the oracle, in place
    and out of place, at the tile edges of the one-launch shapes."""
    from paper_cs_0004013_amd import binding
    torch = torch_cuda()
    rng = np.random.default_rng(21)
    with binding.Server(hbm_budget_bytes=1 << 28, num_streams=2, alone_min_keys=1 << 16) as srv:
        for n in (1, 2, 63, 2047, 2048, 2049, 8192, 8193, 16383, 16384, 16385, 40_000):
            for inplace in (False, True):
                announce(f"server lone request n={n} inplace={inplace}")
                keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
                src = torch.from_numpy(keys.view(np.int32)).to("cuda")
                out = src if inplace else torch.empty_like(src)
                spl = torch.empty(63, dtype=torch.int32, device="cuda")
                tk = srv.submit_ptr(src.data_ptr(), out.data_ptr(), n, 64, spl.data_ptr())
                assert srv.wait(tk) == AP_OK
                torch.cuda.synchronize()
                w = oracle.sort_u32(keys)
                assert np.array_equal(to_host(out), w)
                assert np.array_equal(to_host(spl), oracle.splitters(w, 64))


def test_pass_shape_changed_while_queued():
    """A long request admitted under one pass tile shape and launched after the shape changed: its
    reserved scratch may no longer hold the layout, and then it fails on its own (AP_ERR_DEVICE)
    rather than writing past its range; otherwise it completes correctly.  The request running
    beside it and a later one are unaffected."""
    from paper_cs_0004013_amd import binding
    torch = torch_cuda()
    pool = Pool(1 << 24)
    with binding.Server(hbm_budget_bytes=1 << 30, num_streams=1, alone_min_keys=1 << 16) as srv:
        try:
            binding.ap_set_pass_shape(3)
            a_out = torch.empty(1 << 24, dtype=torch.int32, device="cuda")
            b_out = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
            announce("server: pass shape changed while a request is queued")
            ta = srv.submit(pool.dev["a"], a_out, 64)                    # occupies the only slot
            t0 = time.monotonic()
            while srv.stats()["alone"] < 1 and time.monotonic() - t0 < 10.0:
                pass                                                     # until it has launched
            tb = srv.submit(pool.dev["b"][:1 << 20], b_out, 64)          # admitted under shape 3
            binding.ap_set_pass_shape(0)                                 # 4K tiles: a larger layout
            assert srv.wait(ta) == AP_OK
            st_b = srv.wait(tb)
        finally:
            binding.ap_set_pass_shape(-1)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(a_out), oracle.sort_u32(pool.host["a"]))
        assert st_b in (AP_OK, AP_ERR_DEVICE)
        if st_b == AP_OK:
            assert np.array_equal(to_host(b_out), oracle.sort_u32(pool.host["b"][:1 << 20]))
        c_out = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
        assert srv.wait(srv.submit(pool.dev["c"][:1 << 20], c_out, 64)) == AP_OK
        torch.cuda.synchronize()
        assert np.array_equal(to_host(c_out), oracle.sort_u32(pool.host["c"][:1 << 20]))


def test_destroy_cancels_queued():
    from paper_cs_0004013_amd import binding
    torch = torch_cuda()
    pool = Pool(1 << 22)
    srv = binding.Server(hbm_budget_bytes=1 << 30, num_streams=1, alone_min_keys=1 << 20)
    outs = []
    for i in range(6):
        src = pool.dev["a"][:1 << 22]
        out = torch.empty(1 << 22, dtype=torch.int32, device="cuda")
        outs.append(out)
        srv.submit(src, out, 64)
    srv.close()                                   # running one finishes, queued ones are cancelled
    torch.cuda.synchronize()
