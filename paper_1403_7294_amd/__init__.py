"""Aho-Corasick multi-pattern matching on MI355X (gfx950).

A thin ctypes binding over the C ABI of ``libac.so`` (declared in
``include/ac.h``): the functions below carry the ABI's names and only
marshal arguments.  Every step of the scan runs in the library's HIP
kernels; PyTorch provides device memory (tensors) and streams.  If the
library is not built the first call raises ``LibraryMissing``: there is no
CPU fallback.

    d = ac_build(patterns, sigma=4)             # stage 1 (host), handle
    out, total = scan(d, text_u8_or_packed, fmt)  # stage 2 (GPU)
    ac_destroy(d)

``patterns`` is a list of code sequences, or any object with ``symbols`` and
``offsets`` (CSR, offsets of length count+1).
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libac.so")

AC_OK = 0
AC_E_INVALID = -1
AC_E_EMPTY_PATTERN = -2
AC_E_SYMBOL = -3
AC_E_TOO_LARGE = -4
AC_E_NOMEM = -5
AC_E_OVERFLOW = -6
AC_E_HIP = -7
AC_E_NO_DEVICE = -8
AC_E_TIMEOUT = -9

AC_TEXT_U8 = 0
AC_TEXT_2BIT = 1
AC_ALPHA_DNA = 0
AC_ALPHA_PROTEIN = 1
AC_PLACE_AUTO, AC_PLACE_LDS, AC_PLACE_GLOBAL, AC_PLACE_HYBRID, AC_PLACE_LDS2, AC_PLACE_LDS16 = \
    0, 1, 2, 3, 4, 5
AC_BUILD_HOST_ONLY = 1
AC_BUILD_SERIAL = 2
AC_SEGMENT = 64
AC_DENSE_SEGMENT_MATCHES = 256

# every symbol include/ac.h declares
ABI_SYMBOLS = [
    "ac_build", "ac_destroy", "ac_dict_get_info", "ac_debug_export", "ac_encode",
    "ac_scan_workspace_size", "ac_scan", "ac_batch_create", "ac_batch_run",
    "ac_batch_destroy", "ac_scan_batch", "ac_status_str", "ac_device_info",
    "ac_timing_enable", "ac_timing_read", "ac_build_partitioned", "ac_dict_parts",
    "ac_scan_pfac", "ac_sort_workspace_size", "ac_sort_matches", "ac_scan_noalloc",
    "ac_scan_batch_workspace_size", "ac_server_create", "ac_server_submit", "ac_server_wait",
    "ac_server_release", "ac_server_request_charge", "ac_server_stats", "ac_server_destroy",
]
AC_SORT_BY_END = 1
AC_NOALLOC_MAX_WORKSPACE = 64 << 20
(AC_K_ENCODE, AC_K_COUNT, AC_K_OFFSETS, AC_K_SCATTER, AC_K_EMIT, AC_K_TOTALS, AC_K_EMIT_DENSE,
 AC_K_PFAC, AC_K_SORT) = range(9)
AC_K_KINDS = 9
AC_TIMING_ALL = 1


def AC_TIMING_KIND(k: int) -> int:
    return 2 << k


KERNEL_NAMES = ["encode", "count", "offsets", "scatter", "emit", "totals", "emit_dense", "pfac",
                "sort"]


class LibraryMissing(RuntimeError):
    pass


class ACError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = _lib_status(status)
        super().__init__(f"{where}: {msg} ({status})" if where else f"{msg} ({status})")


class ac_match(ctypes.Structure):
    _fields_ = [("pattern_id", ctypes.c_uint32), ("end_pos", ctypes.c_uint32)]


class ac_build_opts(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_uint32), ("placement", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("hot_states", ctypes.c_uint32)]


class ac_dict_info(ctypes.Structure):
    _fields_ = [("states", ctypes.c_uint32), ("patterns", ctypes.c_uint32),
                ("sigma", ctypes.c_uint32), ("min_len", ctypes.c_uint32),
                ("max_len", ctypes.c_uint32), ("first_output_state", ctypes.c_uint32),
                ("max_output", ctypes.c_uint32), ("placement", ctypes.c_uint32),
                ("hot_states", ctypes.c_uint32), ("has_device", ctypes.c_uint32),
                ("output_entries", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64),
                ("build_ms", ctypes.c_double)]


class ac_tune(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint32), ("block_threads", ctypes.c_uint32),
                ("placement", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("chains", ctypes.c_uint32)]


class ac_server_opts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("staging_bytes", ctypes.c_uint64),
                ("max_batch", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("copy_threads", ctypes.c_uint32), ("max_wait_us", ctypes.c_uint32),
                ("fail_batch", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("margin", ctypes.c_double), ("tune", ac_tune)]


class ac_server_counters(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("bases", ctypes.c_uint64),
                ("matches", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("reruns", ctypes.c_uint64), ("overlapped", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64),
                ("wall_s", ctypes.c_double), ("failed", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ac_batch_item(ctypes.Structure):
    _fields_ = [("dict", ctypes.c_void_p), ("d_text", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("fmt", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("d_out", ctypes.c_void_p), ("capacity", ctypes.c_uint64),
                ("d_count", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libac.so (raises LibraryMissing if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} is not built; run `python -m paper_1403_7294_amd.build`")
    # torch ships its own HIP runtime under the same soname as the system's;
    # loading torch first makes the library bind to that one, so the process
    # has a single HIP runtime whichever package touches the GPU first
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, u32, u64, i = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.ac_build.argtypes = [P, P, u32, ctypes.POINTER(ac_build_opts), ctypes.POINTER(P)]
    L.ac_build.restype = i
    L.ac_destroy.argtypes = [P]
    L.ac_destroy.restype = None
    L.ac_dict_get_info.argtypes = [P, ctypes.POINTER(ac_dict_info)]
    L.ac_dict_get_info.restype = i
    L.ac_debug_export.argtypes = [P, P, P, P, P]
    L.ac_debug_export.restype = i
    L.ac_encode.argtypes = [P, u64, u32, u32, P, P, P]
    L.ac_encode.restype = i
    L.ac_scan_workspace_size.argtypes = [P, u64, u32, ctypes.POINTER(ac_tune),
                                         ctypes.POINTER(u64)]
    L.ac_scan_workspace_size.restype = i
    L.ac_scan.argtypes = [P, P, u64, u32, P, u64, P, ctypes.POINTER(ac_tune), P, u64, P]
    L.ac_scan.restype = i
    L.ac_server_create.argtypes = [P, u32, ctypes.POINTER(ac_server_opts), ctypes.POINTER(P)]
    L.ac_server_submit.argtypes = [P, P, u64, u32, ctypes.POINTER(u64)]
    L.ac_server_wait.argtypes = [P, u64, ctypes.c_int64, ctypes.POINTER(ctypes.POINTER(ac_match)),
                                 ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double)]
    L.ac_server_release.argtypes = [P, u64]
    L.ac_server_request_charge.argtypes = [P, u64, u32, ctypes.POINTER(u64)]
    L.ac_server_stats.argtypes = [P, ctypes.POINTER(ac_server_counters), P, u64]
    L.ac_server_destroy.argtypes = [P]
    for name in ("ac_server_create", "ac_server_submit", "ac_server_wait", "ac_server_release",
                 "ac_server_request_charge", "ac_server_stats", "ac_server_destroy"):
        getattr(L, name).restype = i
    L.ac_scan_noalloc.argtypes = [P, P, u64, u32, P, u64, P, ctypes.POINTER(ac_tune), P]
    L.ac_scan_noalloc.restype = i
    L.ac_batch_create.argtypes = [ctypes.POINTER(ac_batch_item), u32, ctypes.POINTER(ac_tune),
                                  ctypes.POINTER(P)]
    L.ac_batch_create.restype = i
    L.ac_batch_run.argtypes = [P, P]
    L.ac_batch_run.restype = i
    L.ac_batch_destroy.argtypes = [P]
    L.ac_batch_destroy.restype = None
    L.ac_scan_batch.argtypes = [ctypes.POINTER(ac_batch_item), u32, ctypes.POINTER(ac_tune), P,
                                u64, P]
    L.ac_scan_batch_workspace_size.argtypes = [ctypes.POINTER(ac_batch_item), u32,
                                               ctypes.POINTER(ac_tune), ctypes.POINTER(u64)]
    L.ac_scan_batch_workspace_size.restype = i
    L.ac_scan_batch.restype = i
    L.ac_status_str.argtypes = [i]
    L.ac_status_str.restype = ctypes.c_char_p
    L.ac_device_info.argtypes = [ctypes.POINTER(u32), ctypes.POINTER(u32)]
    L.ac_device_info.restype = i
    L.ac_timing_enable.argtypes = [i]
    L.ac_timing_enable.restype = i
    L.ac_timing_read.argtypes = [P, P, i]
    L.ac_timing_read.restype = i
    L.ac_build_partitioned.argtypes = [P, P, u32, ctypes.POINTER(ac_build_opts), u32,
                                       ctypes.POINTER(P)]
    L.ac_build_partitioned.restype = i
    L.ac_dict_parts.argtypes = [P, ctypes.POINTER(u32), P]
    L.ac_dict_parts.restype = i
    L.ac_scan_pfac.argtypes = [P, P, u64, u32, P, u64, P, P]
    L.ac_scan_pfac.restype = i
    L.ac_sort_workspace_size.argtypes = [u64, ctypes.POINTER(u64)]
    L.ac_sort_workspace_size.restype = i
    L.ac_sort_matches.argtypes = [P, u64, u32, u32, P, u64, P]
    L.ac_sort_matches.restype = i
    _lib = L
    return L


def _lib_status(s: int) -> str:
    try:
        return lib().ac_status_str(s).decode()
    except LibraryMissing:
        return "status"


def _check(rc: int, where: str):
    if rc != AC_OK:
        raise ACError(rc, where)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _tune(t) -> Optional[ac_tune]:
    if t is None:
        return None
    if isinstance(t, ac_tune):
        return t
    return ac_tune(t.get("chunk", 0), t.get("block_threads", 0), t.get("placement", 0),
                   t.get("blocks_per_cu", 0), t.get("chains", 0))


def _tune_ref(t):
    t = _tune(t)
    return ctypes.byref(t) if t is not None else None


def _csr(patterns) -> Tuple[np.ndarray, np.ndarray]:
    if hasattr(patterns, "symbols") and hasattr(patterns, "offsets"):
        sym = np.ascontiguousarray(patterns.symbols, dtype=np.uint8)
        off = np.ascontiguousarray(patterns.offsets, dtype=np.uint64)
    else:
        lens = [len(p) for p in patterns]
        off = np.zeros(len(lens) + 1, dtype=np.uint64)
        np.cumsum(lens, out=off[1:])
        parts = [np.asarray(p, dtype=np.uint8) for p in patterns]
        sym = np.concatenate(parts) if off[-1] else np.zeros(0, dtype=np.uint8)
    if sym.size == 0:
        sym = np.zeros(1, dtype=np.uint8)
    return sym, off


# ------------------------------------------------------------------ ABI calls

def ac_build(patterns, sigma: int = 4, placement: int = AC_PLACE_AUTO, host_only: bool = False,
             hot_states: int = 0, serial: bool = False) -> "Dict":
    """Stage 1: compile patterns (paper section III.A) into a dictionary."""
    sym, off = _csr(patterns)
    flags = (AC_BUILD_HOST_ONLY if host_only else 0) | (AC_BUILD_SERIAL if serial else 0)
    opts = ac_build_opts(sigma, placement, flags, hot_states)
    h = ctypes.c_void_p()
    _check(lib().ac_build(sym.ctypes.data, off.ctypes.data, len(off) - 1, ctypes.byref(opts),
                          ctypes.byref(h)), "ac_build")
    return Dict(h)


def ac_build_partitioned(patterns, sigma: int = 4, parts: int = 0, placement: int = AC_PLACE_AUTO,
                         host_only: bool = False) -> "Dict":
    """The paper's second design: one machine per contiguous pattern slice
    (parts = 0: the fewest slices whose tables fit LDS)."""
    sym, off = _csr(patterns)
    opts = ac_build_opts(sigma, placement, AC_BUILD_HOST_ONLY if host_only else 0, 0)
    h = ctypes.c_void_p()
    _check(lib().ac_build_partitioned(sym.ctypes.data, off.ctypes.data, len(off) - 1,
                                      ctypes.byref(opts), parts, ctypes.byref(h)),
           "ac_build_partitioned")
    return Dict(h)


def ac_dict_parts(d: "Dict") -> List[int]:
    """First pattern id of each slice ([] for an ordinary dictionary)."""
    k = ctypes.c_uint32()
    _check(lib().ac_dict_parts(d.handle, ctypes.byref(k), None), "ac_dict_parts")
    ids = (ctypes.c_uint32 * max(1, k.value))()
    _check(lib().ac_dict_parts(d.handle, ctypes.byref(k), ids), "ac_dict_parts")
    return list(ids[:k.value])


def ac_scan_pfac(d: "Dict", text_dev, n: int, fmt: int, out_dev, capacity: int, count_dev,
                 stream=None) -> None:
    """Failure-less scan (one thread per start position); same results as ac_scan."""
    _check(lib().ac_scan_pfac(d.handle, text_dev.data_ptr() if n else None, n, fmt,
                              out_dev.data_ptr() if capacity else None, capacity,
                              count_dev.data_ptr(), _stream_ptr(stream)), "ac_scan_pfac")


def ac_sort_workspace_size(n: int) -> int:
    b = ctypes.c_uint64()
    _check(lib().ac_sort_workspace_size(n, ctypes.byref(b)), "ac_sort_workspace_size")
    return b.value


def ac_sort_matches(matches_dev, n: int, flags: int = 0, end_bits: int = 0, workspace_dev=None,
                    stream=None) -> None:
    """Sort (M, 2) int32 match records in place into (end, id) order."""
    ws = workspace_dev.data_ptr() if workspace_dev is not None else None
    wsb = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().ac_sort_matches(matches_dev.data_ptr() if n else None, n, flags, end_bits, ws,
                                 wsb, _stream_ptr(stream)), "ac_sort_matches")


def ac_destroy(d: "Dict") -> None:
    d.close()


def ac_dict_get_info(d: "Dict") -> ac_dict_info:
    info = ac_dict_info()
    _check(lib().ac_dict_get_info(d.handle, ctypes.byref(info)), "ac_dict_get_info")
    return info


def ac_debug_export(d: "Dict"):
    """Host copies of the compiled tables: (delta[S, sigma], out_off, out_ids, depth)."""
    info = ac_dict_get_info(d)
    S, sig = info.states, info.sigma
    delta = np.empty(S * sig, dtype=np.uint32)
    out_off = np.empty(S - info.first_output_state + 1, dtype=np.uint32)
    out_ids = np.empty(max(1, info.output_entries), dtype=np.uint32)
    depth = np.empty(S, dtype=np.uint32)
    _check(lib().ac_debug_export(d.handle, delta.ctypes.data, out_off.ctypes.data,
                                 out_ids.ctypes.data, depth.ctypes.data), "ac_debug_export")
    return delta.reshape(S, sig), out_off, out_ids[:info.output_entries], depth


def ac_encode(ascii_dev, alphabet: int, fmt: int, out_dev, invalid_dev=None, stream=None) -> None:
    """Letters -> codes on the GPU (torch uint8 tensors)."""
    _check(lib().ac_encode(ascii_dev.data_ptr(), ascii_dev.numel(), alphabet, fmt,
                           out_dev.data_ptr(),
                           invalid_dev.data_ptr() if invalid_dev is not None else None,
                           _stream_ptr(stream)), "ac_encode")


def ac_scan_workspace_size(d: "Dict", n: int, fmt: int, tune=None) -> int:
    b = ctypes.c_uint64()
    _check(lib().ac_scan_workspace_size(d.handle, n, fmt, _tune_ref(tune), ctypes.byref(b)),
           "ac_scan_workspace_size")
    return b.value


def ac_scan(d: "Dict", text_dev, n: int, fmt: int, out_dev, capacity: int, count_dev,
            tune=None, workspace_dev=None, stream=None) -> None:
    """Stage 2 on the GPU; stream-ordered, returns after enqueueing."""
    ws = workspace_dev.data_ptr() if workspace_dev is not None else None
    wsb = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().ac_scan(d.handle, text_dev.data_ptr() if n else None, n, fmt,
                         out_dev.data_ptr() if capacity else None, capacity,
                         count_dev.data_ptr(), _tune_ref(tune), ws, wsb,
                         _stream_ptr(stream)), "ac_scan")


def ac_scan_noalloc(d: "Dict", text_dev, n: int, fmt: int, out_dev, capacity: int, count_dev,
                    tune=None, stream=None) -> None:
    """ac_scan with the library's own device scratch array as workspace: no
    memory is allocated (see AC_NOALLOC_MAX_WORKSPACE)."""
    _check(lib().ac_scan_noalloc(d.handle, text_dev.data_ptr() if n else None, n, fmt,
                                 out_dev.data_ptr() if capacity else None, capacity,
                                 count_dev.data_ptr(), _tune_ref(tune), _stream_ptr(stream)),
           "ac_scan_noalloc")


def _items(items) -> Tuple[ctypes.Array, list]:
    arr = (ac_batch_item * len(items))()
    for i, it in enumerate(items):
        d, text, n, fmt, out, cap, count = it
        arr[i] = ac_batch_item(d.handle, text.data_ptr() if n else None, n, fmt, 0,
                               out.data_ptr() if cap else None, cap, count.data_ptr())
    return arr, list(items)


def ac_scan_batch(items: Sequence[tuple], tune=None, stream=None, workspace_dev=None) -> None:
    """items: (dict, text_dev, n, fmt, out_dev, capacity, count_dev) tuples.
    workspace_dev: device buffer of ac_scan_batch_workspace_size(items) bytes,
    or None for the library's stream-ordered allocation."""
    arr, _ = _items(items)
    ws = workspace_dev.data_ptr() if workspace_dev is not None else None
    wsb = workspace_dev.numel() * workspace_dev.element_size() if workspace_dev is not None else 0
    _check(lib().ac_scan_batch(arr, len(items), _tune_ref(tune), ws, wsb, _stream_ptr(stream)),
           "ac_scan_batch")


def ac_scan_batch_workspace_size(items: Sequence[tuple], tune=None) -> int:
    arr, _ = _items(items)
    b = ctypes.c_uint64()
    _check(lib().ac_scan_batch_workspace_size(arr, len(items), _tune_ref(tune), ctypes.byref(b)),
           "ac_scan_batch_workspace_size")
    return b.value


# ac_batch_item as a numpy record (same layout as the C struct), so that a
# caller can fill a whole batch's descriptors with array operations
BATCH_ITEM_DTYPE = np.dtype([("dict", "<u8"), ("text", "<u8"), ("n", "<u8"), ("fmt", "<u4"),
                             ("reserved", "<u4"), ("out", "<u8"), ("capacity", "<u8"),
                             ("count", "<u8")], align=True)


def ac_scan_batch_records(records: np.ndarray, tune=None, workspace_ptr=None,
                          workspace_bytes: int = 0, stream=None) -> None:
    """ac_scan_batch over a BATCH_ITEM_DTYPE array (device pointers as ints)."""
    assert records.dtype == BATCH_ITEM_DTYPE and records.flags.c_contiguous
    _check(lib().ac_scan_batch(records.ctypes.data_as(ctypes.POINTER(ac_batch_item)),
                               len(records), _tune_ref(tune), workspace_ptr, workspace_bytes,
                               _stream_ptr(stream)), "ac_scan_batch")


def ac_scan_batch_records_workspace_size(records: np.ndarray, tune=None) -> int:
    assert records.dtype == BATCH_ITEM_DTYPE and records.flags.c_contiguous
    b = ctypes.c_uint64()
    _check(lib().ac_scan_batch_workspace_size(
        records.ctypes.data_as(ctypes.POINTER(ac_batch_item)), len(records), _tune_ref(tune),
        ctypes.byref(b)), "ac_scan_batch_workspace_size")
    return b.value


def ac_batch_create(items: Sequence[tuple], tune=None) -> "BatchPlan":
    arr, keep = _items(items)
    h = ctypes.c_void_p()
    _check(lib().ac_batch_create(arr, len(items), _tune_ref(tune), ctypes.byref(h)),
           "ac_batch_create")
    return BatchPlan(h, keep)


def ac_batch_run(plan: "BatchPlan", stream=None) -> None:
    _check(lib().ac_batch_run(plan.handle, _stream_ptr(stream)), "ac_batch_run")


def ac_batch_destroy(plan: "BatchPlan") -> None:
    plan.close()


def ac_status_str(status: int) -> str:
    return lib().ac_status_str(status).decode()


def ac_device_info() -> Tuple[int, int]:
    cu, lds = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().ac_device_info(ctypes.byref(cu), ctypes.byref(lds)), "ac_device_info")
    return cu.value, lds.value


def ac_timing_enable(on, kinds=None) -> None:
    """on: True/False for every kernel kind; kinds: an iterable of AC_K_*
    values to time only those."""
    v = 1 if on else 0
    if on and kinds is not None:
        v = 0
        for k in kinds:
            v |= AC_TIMING_KIND(k)
    _check(lib().ac_timing_enable(v), "ac_timing_enable")


def ac_timing_read(reset: bool = False):
    """{kernel name: (total ms, launches)} since the last reset."""
    ms = (ctypes.c_double * AC_K_KINDS)()
    n = (ctypes.c_uint64 * AC_K_KINDS)()
    _check(lib().ac_timing_read(ms, n, 1 if reset else 0), "ac_timing_read")
    return {KERNEL_NAMES[k]: (ms[k], n[k]) for k in range(AC_K_KINDS)}


# ------------------------------------------------------------------ handles

class Dict:
    """Owning wrapper of an ac_dict*; freed by close() or garbage collection."""

    def __init__(self, handle: ctypes.c_void_p):
        self.handle = handle
        self.info = ac_dict_get_info(self)

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().ac_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep  # the tensors the plan points at

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().ac_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ helpers

def text_symbols(text_dev, fmt: int, n: Optional[int] = None) -> int:
    if n is not None:
        return n
    return text_dev.numel() * (4 if fmt == AC_TEXT_2BIT else 1)


def scan(d: Dict, text_dev, fmt: int = AC_TEXT_U8, n: Optional[int] = None, capacity=None,
         tune=None, stream=None):
    """Run ac_scan and return (matches[M, 2] int32 tensor of (pattern_id,
    end_pos) in (end, id) order, total M).  Re-runs once with an exact-size
    buffer when the first guess overflows.  tune="auto" takes the launch
    shape from the autotuner (timed once per shape key, then cached)."""
    import torch
    n = text_symbols(text_dev, fmt, n)
    if isinstance(tune, str):
        if tune != "auto":
            raise ValueError("tune must be None, a dict, an ac_tune or 'auto'")
        from .tune import autotune
        tune = autotune(d, text_dev, n, fmt) if n else None
    dev = text_dev.device
    cap = capacity if capacity is not None else max(1024, n // 4)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev)
    ac_scan(d, text_dev, n, fmt, out, cap, count, tune=tune, stream=stream)
    torch.cuda.current_stream(dev).synchronize() if stream is None else stream.synchronize()
    total = int(count.item())
    if total > cap and capacity is None:
        cap = total
        out = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        ac_scan(d, text_dev, n, fmt, out, cap, count, tune=tune, stream=stream)
        torch.cuda.current_stream(dev).synchronize() if stream is None else stream.synchronize()
    return out[:min(total, cap)], total


def match_keys(matches) -> np.ndarray:
    """(M, 2) (pattern_id, end_pos) -> uint64 keys end << 32 | id (numpy)."""
    m = matches.cpu().numpy().view(np.uint32)
    return (m[:, 1].astype(np.uint64) << np.uint64(32)) | m[:, 0].astype(np.uint64)

