"""ctypes binding of libac_microbench.so: the measured ceilings that the
benchmark divides by (HBM copy, write and read bandwidth, LDS ds_read_b32
rate conflict-free and random, random gathers from L2-sized and larger
tables, dependent-load latency in LDS and in global memory).  Argument
marshalling only; the kernels are in csrc/microbench.hip."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libac_microbench.so")
SYMBOLS = ["acb_hbm_copy", "acb_hbm_write", "acb_hbm_read", "acb_lds_read", "acb_gather",
           "acb_chase"]
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1403_7294_amd.build`")
        try:
            import torch  # noqa: F401  (one HIP runtime per process, as for libac.so)
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, i, d = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_double))
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        L.acb_hbm_copy.argtypes = [P, P, u64, i, d]
        L.acb_hbm_write.argtypes = [P, u64, i, d]
        L.acb_hbm_read.argtypes = [P, u64, i, d]
        L.acb_lds_read.argtypes = [i, u32, i, d, pu64]
        L.acb_gather.argtypes = [P, u64, u32, i, d, pu64]
        L.acb_chase.argtypes = [P, u64, i, u32, i, d]
        for n in SYMBOLS:
            getattr(L, n).restype = i
        _lib = L
    return _lib


def _ok(rc, where):
    if rc != 0:
        raise RuntimeError(f"{where} failed: {rc}")


def _cyclic_permutation(n: int, seed: int) -> np.ndarray:
    """next[] of one random cycle through 0..n-1 (Sattolo's algorithm)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(n).astype(np.int64)
    nxt = np.empty(n, dtype=np.uint32)
    nxt[order] = np.roll(order, -1)
    return nxt


def measure(torch, hbm_bytes: int = 1 << 30, reps: int = 10) -> dict:
    """All ceilings on the current device; each figure in its own unit."""
    L = lib()
    ms = ctypes.c_double()
    cnt = ctypes.c_uint64()
    dev = torch.device("cuda", torch.cuda.current_device())
    a = torch.empty(hbm_bytes, dtype=torch.uint8, device=dev)
    b = torch.empty(hbm_bytes, dtype=torch.uint8, device=dev)
    a.fill_(1)
    res = {"hbm_buffer_bytes": hbm_bytes}
    _ok(L.acb_hbm_copy(b.data_ptr(), a.data_ptr(), hbm_bytes, reps, ctypes.byref(ms)), "copy")
    res["hbm_copy_gbs"] = round(2 * hbm_bytes / (ms.value * 1e-3) / 1e9, 1)
    _ok(L.acb_hbm_write(b.data_ptr(), hbm_bytes, reps, ctypes.byref(ms)), "write")
    res["hbm_write_gbs"] = round(hbm_bytes / (ms.value * 1e-3) / 1e9, 1)
    _ok(L.acb_hbm_read(a.data_ptr(), hbm_bytes, reps, ctypes.byref(ms)), "read")
    res["hbm_read_gbs"] = round(hbm_bytes / (ms.value * 1e-3) / 1e9, 1)
    del a, b
    for name, rnd in (("lds_read_conflict_free", 0), ("lds_read_random", 1)):
        _ok(L.acb_lds_read(rnd, 4096, reps, ctypes.byref(ms), ctypes.byref(cnt)), name)
        res[name + "_per_s"] = round(cnt.value / (ms.value * 1e-3), 1)
    for mib in (2, 8, 64):
        entries = (mib << 20) // 4
        t = torch.randint(0, 1 << 30, (entries,), dtype=torch.int32, device=dev)
        _ok(L.acb_gather(t.data_ptr(), entries, 256, reps, ctypes.byref(ms), ctypes.byref(cnt)),
            "gather")
        res[f"gather_{mib}mib_per_s"] = round(cnt.value / (ms.value * 1e-3), 1)
        del t
    lat = ctypes.c_double()
    nxt = torch.from_numpy(_cyclic_permutation(16384, 1).view(np.int32)).to(dev)
    _ok(L.acb_chase(nxt.data_ptr(), 16384, 1, 20000, 3, ctypes.byref(lat)), "chase lds")
    res["lds_dependent_load_ns"] = round(lat.value, 2)
    for mib in (2, 64):
        entries = (mib << 20) // 4
        nxt = torch.from_numpy(_cyclic_permutation(entries, 2).view(np.int32)).to(dev)
        _ok(L.acb_chase(nxt.data_ptr(), entries, 0, 20000, 3, ctypes.byref(lat)), "chase")
        res[f"global_dependent_load_{mib}mib_ns"] = round(lat.value, 2)
    return res
