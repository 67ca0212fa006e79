"""ctypes binding of libapsort.so (include/apsort.h), same names as the C ABI.

Argument marshalling only: every step of the sort runs in the library's HIP kernels.  Tensors are
torch CUDA (HIP) tensors of dtype int32 or uint32 (keys are reinterpreted bit for bit as uint32);
the stream is torch's current stream unless one is given.  PyTorch provides device memory and
streams, nothing else.  There is no fallback: a missing library or a failed call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapsort.so")
TUNE_TABLE = os.path.join(HERE, "tune_gfx950.txt")   # written by paper_cs_0004013_amd.autotune

AP_OK = 0
STATUS = {0: "AP_OK", 1: "AP_ERR_INVALID", 2: "AP_ERR_NOMEM", 3: "AP_ERR_HIP", 4: "AP_ERR_BUDGET",
          5: "AP_ERR_QUEUE_FULL", 6: "AP_ERR_TIMEOUT", 7: "AP_ERR_DEVICE", 8: "AP_ERR_CANCELLED"}
MAX_KEYS = 1 << 30

class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("num_streams", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("max_queue", ctypes.c_int), ("alone_min_keys", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("submitted", "completed", "failed", "cancelled", "batches", "alone",
                                              "keys", "latency_samples")] + \
               [(f, ctypes.c_double) for f in ("p50_us", "p99_us", "mean_us", "max_us", "queue_p50_us",
                                              "queue_p99_us")] + \
               [(f, ctypes.c_uint64) for f in ("scratch_budget_bytes", "scratch_peak_bytes")]


# (name, restype, argtypes) of every exported entry point
_VP, _SZ, _I, _U64P = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)
SIGNATURES = [
    ("ap_sort_u32", _I, [_VP, _VP, _SZ, _I, _VP, _VP]),
    ("ap_sort_workspace_bytes", _SZ, [_SZ]),
    ("ap_workspace_init", _I, [_VP, _SZ, _VP]),
    ("ap_sort_u32_ws", _I, [_VP, _VP, _SZ, _I, _VP, _VP, _SZ, _VP]),
    ("ap_sort_u32_noalloc", _I, [_VP, _VP, _SZ, _I, _VP, _VP]),
    ("ap_sort_u32_msd", _I, [_VP, _VP, _SZ, _I, _VP, _VP]),
    ("ap_sort_pairs_u32", _I, [_VP, _VP, _VP, _VP, _SZ, _I, _VP, _VP]),
    ("ap_sort_pairs_workspace_bytes", _SZ, [_SZ]),
    ("ap_sort_pairs_u32_ws", _I, [_VP, _VP, _VP, _VP, _SZ, _I, _VP, _VP, _SZ, _VP]),
    ("ap_merge_u32", _I, [_VP, _SZ, _VP, _SZ, _VP, _VP]),
    ("ap_merge_adjacent_u32", _I, [_VP, _SZ, _SZ, _VP]),
    ("ap_digit_plan_u32", _I, [_VP, _SZ, _I, _VP, _VP, _VP]),
    ("ap_release_cache", _I, []),
    ("ap_check_u32", _I, [_VP, _SZ, _VP, _VP]),
    ("ap_check_u32_batch", _I, [_VP, _VP, _I, _SZ, _VP, _VP]),
    ("ap_profile_enable", _I, [_I]),
    ("ap_profile_read", _I, [ctypes.POINTER(ctypes.c_double), _U64P, _I]),
    ("ap_sort_u32_segmented", _I, [_VP, _SZ, _VP, _I, _VP, _VP]),
    ("ap_segmented_workspace_bytes", _SZ, [_SZ, _I]),
    ("ap_segmented_set_long_min", _I, [_SZ]),
    ("ap_segmented_get_long_min", _SZ, []),
    ("ap_segmented_num_configs", _I, []),
    ("ap_segmented_num_groups", _I, []),
    ("ap_segmented_config_info", _I, [_I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    ("ap_segmented_set_config", _I, [_I]),
    ("ap_segmented_set_group", _I, [_I, _I, _I, _I]),
    ("ap_segmented_get_group", _I, [_I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    ("ap_load_tuning", _I, [ctypes.c_char_p]),
    ("ap_server_create", _I, [ctypes.POINTER(ServerCfg), ctypes.POINTER(_VP)]),
    ("ap_server_submit", _I, [_VP, _VP, _VP, _SZ, _I, _VP, _U64P]),
    ("ap_server_submit_flags", _I, [_VP, _VP, _VP, _SZ, _I, _VP, ctypes.c_uint, _U64P]),
    ("ap_server_submit_at", _I, [_VP, _VP, _VP, _SZ, _I, _VP, ctypes.c_uint, ctypes.c_uint64, _U64P]),
    ("ap_server_wait", _I, [_VP, ctypes.c_uint64, ctypes.c_int64]),
    ("ap_server_poll", _I, [_VP, ctypes.c_uint64]),
    ("ap_server_get_stats", _I, [_VP, ctypes.POINTER(ServerStats), _I]),
    ("ap_server_destroy", _I, [_VP]),
    ("ap_rank_check_state", _I, []),
    ("ap_set_rank_mode", _I, [_I]),
    ("ap_set_pass_shape", _I, [_I]),
    ("ap_debug_pass", _I, [_I, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t]),
    ("ap_last_error", ctypes.c_char_p, []),
    ("ap_version", ctypes.c_char_p, []),
]


class ApError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Open libapsort.so (raises if it has not been built).

    PyTorch is imported first.  It bundles its own HIP runtime under the soname the library
    links (libamdhip64.so.7), but asks for it by another name, so the dynamic loader shares one
    runtime only when torch's copy is already loaded: opened the other way round, the process
    would hold two HIP runtimes, and the second one to start finds no device."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_cs_0004013_amd.build` "
                               "(or __graft_entry__.build()) first")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if os.path.exists(TUNE_TABLE):
            st = L.ap_load_tuning(TUNE_TABLE.encode())
            if st != AP_OK:
                raise ApError(st, "ap_load_tuning", L.ap_last_error().decode(errors="replace"))
        _lib = L
    return _lib


def last_error() -> str:
    return lib().ap_last_error().decode(errors="replace")


def check(status: int, where: str) -> None:
    if status != AP_OK:
        raise ApError(status, where, last_error())


def _torch():
    import torch
    return torch


def _keys_ptr(t, name: str) -> int:
    torch = _torch()
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"{name}: int32/uint32 tensor expected, got {t.dtype}")
    if not t.is_cuda:
        raise TypeError(f"{name}: device tensor expected")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int:
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def ap_sort_u32(t_in, t_out, P: int = 64, t_splitters=None, stream=None) -> None:
    """Sort t_in into t_out (may be the same tensor) and write the P-1 splitters (A1-A7)."""
    n = t_in.numel()
    if t_out.numel() != n:
        raise ValueError("input and output sizes differ")
    spl = 0
    if t_splitters is not None:
        if t_splitters.numel() < max(P - 1, 0):
            raise ValueError("splitter tensor needs P-1 entries")
        spl = _keys_ptr(t_splitters, "splitters")
    st = lib().ap_sort_u32(_keys_ptr(t_in, "in") if n else None, _keys_ptr(t_out, "out") if n else None, n, P,
                           spl or None, _stream(stream))
    check(st, "ap_sort_u32")


def ap_sort_u32_msd(t_in, t_out, P: int = 64, t_splitters=None, stream=None) -> None:
    """ap_sort_u32 as bucketing on the top 16 bits, then a local sort of every bucket."""
    n = t_in.numel()
    if t_out.numel() != n:
        raise ValueError("input and output sizes differ")
    spl = None
    if t_splitters is not None:
        if t_splitters.numel() < max(P - 1, 0):
            raise ValueError("splitter tensor needs P-1 entries")
        spl = _keys_ptr(t_splitters, "splitters")
    st = lib().ap_sort_u32_msd(_keys_ptr(t_in, "in") if n else None, _keys_ptr(t_out, "out") if n else None, n, P,
                               spl, _stream(stream))
    check(st, "ap_sort_u32_msd")


NOALLOC_MAX_KEYS = 1 << 22


def ap_sort_u32_noalloc(t_in, t_out, P: int = 64, t_splitters=None, stream=None) -> None:
    """ap_sort_u32 with the library's fixed scratch array (no allocation); n <= 2^22."""
    n = t_in.numel()
    if t_out.numel() != n:
        raise ValueError("input and output sizes differ")
    spl = None
    if t_splitters is not None:
        if t_splitters.numel() < max(P - 1, 0):
            raise ValueError("splitter tensor needs P-1 entries")
        spl = _keys_ptr(t_splitters, "splitters")
    st = lib().ap_sort_u32_noalloc(_keys_ptr(t_in, "in") if n else None, _keys_ptr(t_out, "out") if n else None, n,
                                   P, spl, _stream(stream))
    check(st, "ap_sort_u32_noalloc")


def ap_sort_pairs_u32(t_keys_in, t_vals_in, t_keys_out, t_vals_out, P: int = 1, t_splitters=None,
                      stream=None) -> None:
    """Sort (key, value) pairs by key; pairs with equal keys keep their input order."""
    n = t_keys_in.numel()
    for t in (t_vals_in, t_keys_out, t_vals_out):
        if t.numel() != n:
            raise ValueError("key and value tensors differ in size")
    spl = None
    if t_splitters is not None:
        if t_splitters.numel() < max(P - 1, 0):
            raise ValueError("splitter tensor needs P-1 entries")
        spl = _keys_ptr(t_splitters, "splitters")
    ptrs = [_keys_ptr(t, name) if n else None for t, name in
            ((t_keys_in, "keys_in"), (t_vals_in, "vals_in"), (t_keys_out, "keys_out"), (t_vals_out, "vals_out"))]
    check(lib().ap_sort_pairs_u32(*ptrs, n, P, spl, _stream(stream)), "ap_sort_pairs_u32")


def ap_sort_pairs_workspace_bytes(n: int) -> int:
    return int(lib().ap_sort_pairs_workspace_bytes(n))


def ap_sort_pairs_u32_ws(t_keys_in, t_vals_in, t_keys_out, t_vals_out, P: int, t_splitters, t_ws,
                         stream=None) -> None:
    n = t_keys_in.numel()
    spl = _keys_ptr(t_splitters, "splitters") if t_splitters is not None else None
    ptrs = [_keys_ptr(t, name) if n else None for t, name in
            ((t_keys_in, "keys_in"), (t_vals_in, "vals_in"), (t_keys_out, "keys_out"), (t_vals_out, "vals_out"))]
    check(lib().ap_sort_pairs_u32_ws(*ptrs, n, P, spl, t_ws.data_ptr(), t_ws.numel() * t_ws.element_size(),
                                     _stream(stream)), "ap_sort_pairs_u32_ws")


def argsort_u32(t_keys, stream=None):
    """(sorted keys, stable sorting permutation) of a uint32-bit int32 tensor, via the pairs sort
    with values 0..n-1."""
    import torch
    n = t_keys.numel()
    idx = torch.arange(n, dtype=torch.int32, device=t_keys.device)
    k_out = torch.empty_like(t_keys)
    perm = torch.empty_like(idx)
    ap_sort_pairs_u32(t_keys, idx, k_out, perm, 1, None, stream)
    return k_out, perm


def ap_merge_u32(t_a, t_b, t_out, stream=None) -> None:
    """Merge two sorted runs into t_out (equal keys: t_a's first)."""
    na, nb = t_a.numel(), t_b.numel()
    if t_out.numel() != na + nb:
        raise ValueError("output size must be len(a) + len(b)")
    check(lib().ap_merge_u32(_keys_ptr(t_a, "a") if na else None, na, _keys_ptr(t_b, "b") if nb else None, nb,
                             _keys_ptr(t_out, "out") if na + nb else None, _stream(stream)), "ap_merge_u32")


def ap_merge_adjacent_u32(t_keys, na: int, stream=None) -> None:
    """Merge the sorted runs t_keys[:na] and t_keys[na:] in place."""
    n = t_keys.numel()
    if not 0 <= na <= n:
        raise ValueError("na out of range")
    check(lib().ap_merge_adjacent_u32(_keys_ptr(t_keys, "keys") if n else None, na, n - na, _stream(stream)),
          "ap_merge_adjacent_u32")


def ap_sort_workspace_bytes(n: int) -> int:
    return int(lib().ap_sort_workspace_bytes(n))


def ap_workspace_init(t_ws, stream=None) -> None:
    check(lib().ap_workspace_init(t_ws.data_ptr(), t_ws.numel() * t_ws.element_size(), _stream(stream)),
          "ap_workspace_init")


def ap_sort_u32_ws(t_in, t_out, P: int, t_splitters, t_ws, stream=None) -> None:
    n = t_in.numel()
    spl = _keys_ptr(t_splitters, "splitters") if t_splitters is not None else None
    st = lib().ap_sort_u32_ws(_keys_ptr(t_in, "in") if n else None, _keys_ptr(t_out, "out") if n else None, n, P,
                              spl, t_ws.data_ptr(), t_ws.numel() * t_ws.element_size(), _stream(stream))
    check(st, "ap_sort_u32_ws")


def ap_digit_plan_u32(t_in, digit_bits: int, t_hist, t_plan=None, stream=None) -> None:
    """Per-digit bucket counts (D x 2^bits) and the pass plan (D run flags + pass count)."""
    n = t_in.numel()
    D = (32 + digit_bits - 1) // digit_bits
    if t_hist.numel() < D << digit_bits:
        raise ValueError("histogram tensor too small")
    if t_plan is not None and t_plan.numel() < D + 1:
        raise ValueError("plan tensor needs D+1 entries")
    st = lib().ap_digit_plan_u32(_keys_ptr(t_in, "in") if n else None, n, digit_bits, _keys_ptr(t_hist, "hist"),
                                 _keys_ptr(t_plan, "plan") if t_plan is not None else None, _stream(stream))
    check(st, "ap_digit_plan_u32")


def ap_check_u32(t_keys, t_acc, n: int | None = None, stream=None) -> None:
    """Accumulate (descents, sum, xor of SplitMix64) of the first n keys into t_acc (3 int64/uint64
    on the device)."""
    n = t_keys.numel() if n is None else n
    if n > t_keys.numel() or t_acc.numel() < 3 or t_acc.element_size() != 8:
        raise ValueError("bad check arguments")
    check(lib().ap_check_u32(_keys_ptr(t_keys, "keys") if n else None, n, t_acc.data_ptr(), _stream(stream)),
          "ap_check_u32")


def ap_check_u32_batch(ptrs_addr: int, counts_addr: int, count: int, max_n: int, acc_addr: int,
                       stream=None) -> None:
    """ap_check_u32 on `count` arrays whose device pointers and key counts are stored in device
    memory at ptrs_addr / counts_addr (uint64 each); results into 3 * count uint64 at acc_addr."""
    check(lib().ap_check_u32_batch(ptrs_addr, counts_addr, count, max_n, acc_addr, _stream(stream)),
          "ap_check_u32_batch")


AP_KIND_HIST, AP_KIND_PASS, AP_KIND_FINAL, AP_KIND_SEG, AP_KIND_MERGE, AP_NKINDS = 0, 1, 9, 10, 11, 16


def ap_profile_enable(on: bool = True) -> None:
    check(lib().ap_profile_enable(1 if on else 0), "ap_profile_enable")


def ap_profile_read() -> tuple[list[float], list[int]]:
    """(milliseconds, launches) per kernel kind since the last read; waits for the events."""
    ms = (ctypes.c_double * AP_NKINDS)()
    cnt = (ctypes.c_uint64 * AP_NKINDS)()
    check(lib().ap_profile_read(ms, cnt, AP_NKINDS), "ap_profile_read")
    return list(ms), list(cnt)


def ap_sort_u32_segmented(t_keys, t_offsets, t_status=None, stream=None) -> None:
    """Sort every segment t_keys[t_offsets[s]:t_offsets[s+1]] in place (batched form)."""
    nseg = t_offsets.numel() - 1
    if nseg < 0:
        raise ValueError("offsets need at least one entry")
    n = t_keys.numel()
    st = lib().ap_sort_u32_segmented(_keys_ptr(t_keys, "keys") if n else None, n,
                                     _keys_ptr(t_offsets, "offsets"), nseg,
                                     _keys_ptr(t_status, "status") if t_status is not None else None,
                                     _stream(stream))
    check(st, "ap_sort_u32_segmented")


def ap_segmented_set_long_min(long_min: int) -> None:
    """Segments of at least long_min keys are sorted by device-wide passes (0 = never)."""
    check(lib().ap_segmented_set_long_min(long_min), "ap_segmented_set_long_min")


def ap_segmented_get_long_min() -> int:
    return int(lib().ap_segmented_get_long_min())


def ap_segmented_num_configs() -> int:
    return int(lib().ap_segmented_num_configs())


def ap_segmented_set_config(cfg: int) -> None:
    check(lib().ap_segmented_set_config(cfg), "ap_segmented_set_config")


def ap_segmented_num_groups() -> int:
    return int(lib().ap_segmented_num_groups())


def ap_segmented_config_info(cfg: int) -> tuple[int, int, int]:
    """(digit bits, waves per workgroup, keys per lane) of a compiled-in configuration."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib().ap_segmented_config_info(cfg, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
          "ap_segmented_config_info")
    return a.value, b.value, c.value


def segmented_groups() -> list[tuple[int, int, int]]:
    """Current (cls_lo, cls_hi, cfg) of every length group."""
    out = []
    for g in range(ap_segmented_num_groups()):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().ap_segmented_get_group(g, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "ap_segmented_get_group")
        out.append((a.value, b.value, c.value))
    return out


def set_segmented_groups(groups) -> None:
    """Install (cls_lo, cls_hi, cfg) as groups 0.. in order; the groups not listed become unused."""
    groups = list(groups)
    ng = ap_segmented_num_groups()
    if len(groups) > ng:
        raise ValueError(f"at most {ng} length groups")
    for g in range(ng):
        lo, hi, cfg = groups[g] if g < len(groups) else (1, 0, 0)
        check(lib().ap_segmented_set_group(g, lo, hi, cfg), "ap_segmented_set_group")


def ap_load_tuning(path: str) -> None:
    check(lib().ap_load_tuning(path.encode()), "ap_load_tuning")


AP_SUBMIT_INJECT_FAULT = 1


class Server:
    """Request server (ap_server_*): submit sorts of device buffers, wait on tickets."""

    def __init__(self, hbm_budget_bytes: int = 0, num_streams: int = 0, max_batch: int = 0, max_queue: int = 0,
                 alone_min_keys: int = 0):
        cfg = ServerCfg(hbm_budget_bytes, num_streams, max_batch, max_queue, alone_min_keys)
        h = ctypes.c_void_p()
        check(lib().ap_server_create(ctypes.byref(cfg), ctypes.byref(h)), "ap_server_create")
        self._h = h

    def submit_ptr(self, in_ptr: int, out_ptr: int, n: int, P: int, spl_ptr: int | None = None,
                   flags: int = 0) -> int:
        """Submit by raw device pointers; returns the ticket (raises on rejection)."""
        t = ctypes.c_uint64()
        st = lib().ap_server_submit_flags(self._h, in_ptr or None, out_ptr or None, n, P, spl_ptr or None, flags,
                                          ctypes.byref(t))
        check(st, "ap_server_submit")
        return t.value

    def submit_at_ptr(self, in_ptr: int, out_ptr: int, n: int, P: int, spl_ptr: int | None, arrival_ns: int,
                      flags: int = 0) -> int:
        """Submit a request that arrived at ``arrival_ns`` (time.monotonic_ns(), the clock the server
        measures latency on); its latency is counted from then."""
        t = ctypes.c_uint64()
        st = lib().ap_server_submit_at(self._h, in_ptr or None, out_ptr or None, n, P, spl_ptr or None, flags,
                                       arrival_ns, ctypes.byref(t))
        check(st, "ap_server_submit_at")
        return t.value

    def try_submit_ptr(self, in_ptr: int, out_ptr: int, n: int, P: int, spl_ptr: int | None = None,
                       flags: int = 0) -> tuple[int, int]:
        """(status, ticket) without raising."""
        t = ctypes.c_uint64()
        st = lib().ap_server_submit_flags(self._h, in_ptr or None, out_ptr or None, n, P, spl_ptr or None, flags,
                                          ctypes.byref(t))
        return st, t.value

    def submit(self, t_in, t_out, P: int = 64, t_splitters=None, flags: int = 0) -> int:
        n = t_in.numel()
        return self.submit_ptr(_keys_ptr(t_in, "in") if n else 0, _keys_ptr(t_out, "out") if n else 0, n, P,
                               _keys_ptr(t_splitters, "splitters") if t_splitters is not None else 0, flags)

    def wait(self, ticket: int, timeout_us: int = -1) -> int:
        """Final status of the ticket (AP_OK = 0) or AP_ERR_TIMEOUT (6)."""
        return int(lib().ap_server_wait(self._h, ticket, timeout_us))

    def poll(self, ticket: int) -> int:
        return int(lib().ap_server_poll(self._h, ticket))

    def stats(self, reset_latencies: bool = False) -> dict:
        st = ServerStats()
        check(lib().ap_server_get_stats(self._h, ctypes.byref(st), 1 if reset_latencies else 0), "ap_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self) -> None:
        if self._h:
            check(lib().ap_server_destroy(self._h), "ap_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ap_rank_check_state() -> int:
    return int(lib().ap_rank_check_state())


def ap_set_rank_mode(mode: int) -> None:
    """0 = automatic (atomic rank when the device passed its lane-order check), 1 = mask rank."""
    check(lib().ap_set_rank_mode(mode), "ap_set_rank_mode")


PASS_DBG_NONE, PASS_DBG_PERTURB, PASS_DBG_TRACE = 0, 1, 2
PASS_TRACE_WORDS = 8


def ap_debug_pass(mode: int, seed: int = 0, t_trace=None) -> None:
    """Debug mode of the keys-only digit pass: 0 off, 1 seeded timing perturbation, 2 phase trace
    into t_trace (an int64 device tensor of 8 words per record)."""
    ptr, recs = None, 0
    if t_trace is not None:
        ptr, recs = t_trace.data_ptr(), t_trace.numel() // PASS_TRACE_WORDS
    check(lib().ap_debug_pass(mode, seed, ptr, recs), "ap_debug_pass")


def ap_set_pass_shape(shape: int = -1) -> None:
    """Tile shape of the device-wide digit pass: -1 = by size, 0..3 = 2K/4K/16K/32K keys."""
    check(lib().ap_set_pass_shape(shape), "ap_set_pass_shape")


def ap_release_cache() -> None:
    check(lib().ap_release_cache(), "ap_release_cache")


def ap_version() -> str:
    return lib().ap_version().decode()
