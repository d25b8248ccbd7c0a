"""Autotuner for the scan's launch shape.

The best chunk length, chains per lane, block size and table placement
depend on the dictionary (table size against LDS, match density), the text
size and the text format.  ``autotune`` times a small candidate set with
HIP events on the caller's text and keeps the fastest shape in a JSON cache.
The cache key is (device, format, sigma, states, table bytes, log2 of the
text length), so later scans of similar size reuse the shape without timing.

    from paper_1403_7294_amd import tune
    t = tune.autotune(d, text_dev, n, fmt)      # dict usable as ``tune=``
    out, total = scan(d, text_dev, fmt, n=n, tune=t)

Candidates run the full scan (count, offsets, work list, emit) with an
output buffer of the exact size, so the emit kernels are timed as well.
"""
from __future__ import annotations

import json
import math
import os
import threading
from typing import Dict, List, Optional, Sequence

from . import (AC_PLACE_AUTO, AC_PLACE_GLOBAL, AC_PLACE_HYBRID, AC_PLACE_LDS2, AC_TEXT_2BIT,
               ac_device_info, ac_scan, ac_scan_batch, ac_scan_workspace_size)

CACHE_ENV = "AC_TUNE_CACHE"
_lock = threading.Lock()
_mem: Dict[str, dict] = {}
stats = {"timed": 0, "hits": 0}


def cache_path() -> str:
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_1403_7294_amd", "tune.json")


def _load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    with _lock:
        data = _load()
        data[key] = value
        tmp = p + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
        _mem[key] = value


def key_for(d, n: int, fmt: int) -> str:
    import torch
    name = torch.cuda.get_device_name() if torch.cuda.is_available() else "none"
    i = d.info
    return (f"{name}|fmt{fmt}|s{i.sigma}|S{i.states}|T{i.table_bytes}|"
            f"n2^{int(math.log2(max(n, 1)))}")


def candidates(d, n: int, fmt: int) -> List[Optional[dict]]:
    """Launch shapes worth timing for this dictionary and text."""
    _, lds = ac_device_info()
    fits = d.info.table_bytes + 1024 <= lds - 512
    chunks = (128, 256, 512) if fmt == AC_TEXT_2BIT else (64, 128, 256)
    places = [AC_PLACE_AUTO] if fits else [AC_PLACE_HYBRID, AC_PLACE_GLOBAL]
    if fmt == AC_TEXT_2BIT and d.info.sigma == 4 and d.info.states * 64 <= lds - 512:
        places.append(AC_PLACE_LDS2)
    out: List[Optional[dict]] = [None]  # the library's own choice
    for place in places:
        for chunk in chunks:
            for chains in (1, 2):
                for threads in (512, 1024):
                    out.append({"chunk": chunk, "chains": chains, "block_threads": threads,
                                "placement": place})
    return out


def _time(fn, stream, reps: int) -> float:
    import torch
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def autotune(d, text_dev, n: int, fmt: int, reps: int = 3, cands: Optional[Sequence] = None,
             force: bool = False) -> Optional[dict]:
    """The fastest launch shape for scanning text_dev (n symbols, format fmt)
    with dictionary d; cached by shape key.  Returns a tune dict, or None
    when the library's default is fastest."""
    import torch
    key = key_for(d, n, fmt)
    if not force:
        hit = _mem.get(key) or _load().get(key)
        if hit is not None:
            stats["hits"] += 1
            _mem[key] = hit
            return hit.get("tune")
    dev = text_dev.device
    stream = torch.cuda.current_stream(dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    dummy = torch.empty((1, 2), dtype=torch.int32, device=dev)
    ac_scan(d, text_dev, n, fmt, dummy, 0, count, stream=stream)
    stream.synchronize()
    total = int(count.item())
    out = torch.empty((max(1, total), 2), dtype=torch.int32, device=dev)
    best, best_ms, table = None, float("inf"), []
    for t in (cands if cands is not None else candidates(d, n, fmt)):
        ws = torch.empty(max(1, ac_scan_workspace_size(d, n, fmt, t)), dtype=torch.uint8,
                         device=dev)

        def run():
            ac_scan(d, text_dev, n, fmt, out, total, count, tune=t, workspace_dev=ws,
                    stream=stream)
        ms = _time(run, stream, reps)
        table.append((ms, t))
        if ms < best_ms:
            best, best_ms = t, ms
        del ws
    stats["timed"] += 1
    _store(key, {"tune": best, "ms": round(best_ms, 4),
                 "default_ms": round(table[0][0], 4) if cands is None else None,
                 "candidates": len(table)})
    return best


def autotune_batch(items: Sequence[tuple], reps: int = 3, cands: Optional[Sequence] = None
                   ) -> Optional[dict]:
    """The fastest shared launch shape for one batch (items as for
    ``ac_scan_batch``).  Not cached: batches differ call to call."""
    import torch
    stream = torch.cuda.current_stream()
    fmt = items[0][3]
    chunks = (128, 256, 512) if fmt == AC_TEXT_2BIT else (64, 128, 256)
    if cands is None:
        cands = [None] + [{"chunk": c, "chains": ch, "block_threads": th, "placement": pl}
                          for c in chunks for ch in (1, 2) for th in (512, 1024)
                          for pl in ((AC_PLACE_AUTO, AC_PLACE_LDS2) if fmt == AC_TEXT_2BIT
                                     else (AC_PLACE_AUTO,))]
    best, best_ms = None, float("inf")
    for t in cands:
        ms = _time(lambda: ac_scan_batch(items, tune=t, stream=stream), stream, reps)
        if ms < best_ms:
            best, best_ms = t, ms
    return best
