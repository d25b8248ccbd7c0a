"""Continuous-batching server for Aho-Corasick scans on one GPU.

Python face of the library's serving core (``ac_server_*`` in the C ABI,
``csrc/serve.cpp``).  Requests - a text as letters and the index of one of
the server's device-resident dictionaries - arrive at any time through
``submit``; the core stages their letters in a pinned ring, admits them into
batches while device memory and an in-flight slot allow, runs each batch as
one set of independent scans (the paper's section IV.A) on one of several
streams, so that requests arriving while batches run are admitted at once
and overlap them on the GPU, and hands each request its matches.  A
request's result is its matches as uint64 keys ``end << 32 | pattern_id`` in
(end, id) order: the same as a scan of its text alone.

Queueing, staging, admission, launches and completion all run in the
core's native threads; this module only marshals arguments, so a request
costs the submitting thread one library call and its result one more.
"""
from __future__ import annotations

import concurrent.futures
import ctypes
import dataclasses
import time
from typing import List, Optional, Sequence

import numpy as np

from . import (AC_E_HIP, AC_E_NOMEM, AC_E_SYMBOL, AC_E_TIMEOUT, AC_OK, ACError, ac_build,
               ac_match, ac_server_counters, ac_server_opts, ac_tune, lib)


@dataclasses.dataclass
class ServeStats:
    latencies_s: List[float]
    bases: int
    matches: int
    batches: int
    reruns: int
    wall_s: float
    peak_bytes: int
    overlapped: int = 0   # batches launched while another was in flight
    budget_bytes: int = 0

    def summary(self) -> dict:
        lat = np.array(self.latencies_s) if self.latencies_s else np.zeros(1)
        return {"requests": len(self.latencies_s),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "mean_ms": round(float(lat.mean()) * 1e3, 3),
                "throughput_gbases_s": round(self.bases / self.wall_s / 1e9, 3)
                if self.wall_s else 0.0,
                "requests_per_s": round(len(self.latencies_s) / self.wall_s, 1)
                if self.wall_s else 0.0,
                "matches": self.matches, "batches": self.batches, "reruns": self.reruns,
                "overlapped_batches": self.overlapped,
                "peak_device_bytes": self.peak_bytes, "budget_bytes": self.budget_bytes}


def _error(rc: int) -> Exception:
    if rc == AC_E_NOMEM:
        return MemoryError("request larger than the server's memory budget")
    if rc == AC_E_SYMBOL:
        return ValueError("request text has letters outside ACGTacgt")
    if rc == AC_E_HIP:
        return RuntimeError("server worker failed")
    return ACError(rc, "ac_server_wait")


class ServeFuture:
    """One request's result.  ``result()`` waits for it inside the library
    (without holding the interpreter lock); ``done()`` does not wait."""

    def __init__(self, server: "Server", ticket: int, letters: np.ndarray):
        self._srv = server
        self._ticket = ticket
        self._letters = letters      # the core reads them until they are staged
        self._done = False
        self._res: Optional[np.ndarray] = None
        self._exc: Optional[BaseException] = None
        self.latency_s = 0.0

    def _fetch(self, timeout_us: int) -> bool:
        L = lib()
        ptr = ctypes.POINTER(ac_match)()
        cnt = ctypes.c_uint64()
        lat = ctypes.c_double()
        rc = L.ac_server_wait(self._srv._h, self._ticket, timeout_us, ctypes.byref(ptr),
                              ctypes.byref(cnt), ctypes.byref(lat))
        if rc == AC_E_TIMEOUT:
            return False
        if rc == AC_OK:
            n = cnt.value
            if n:
                m = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctypes.c_uint32)),
                                          shape=(n, 2))
                self._res = ((m[:, 1].astype(np.uint64) << np.uint64(32)) |
                             m[:, 0].astype(np.uint64))
            else:
                self._res = np.zeros(0, dtype=np.uint64)
        else:
            self._exc = _error(rc)
        self.latency_s = lat.value
        L.ac_server_release(self._srv._h, self._ticket)
        self._letters = None
        self._done = True
        return True

    def result(self, timeout: Optional[float] = None):
        if not self._done and not self._fetch(-1 if timeout is None else int(timeout * 1e6)):
            raise concurrent.futures.TimeoutError()
        if self._exc is not None:
            raise self._exc
        return self._res

    def done(self) -> bool:
        return self._done or self._fetch(0)


class Server:
    """Serve scans of DNA texts against dictionaries kept on the GPU.

    dictionaries   list of pattern sets (code lists or CSR objects), DNA codes
    budget_bytes   device memory the server may hold for requests at once
                   (capped by the device's free memory at construction)
    max_batch      requests per batch
    streams        batches in flight at once (>= 2 to overlap)
    staging_bytes  pinned staging ring for letters
    copy_threads   threads that stage letters
    max_wait_us    how long a batch that could grow waits for requests being
                   staged while other batches are in flight
    margin         reserved matches = margin * (mean + 2 sqrt(mean)) + 64
    tune           launch shape of the batches (dict or ac_tune)
    fail_batch     fault injection for tests: the k-th batch's device
                   allocation is reported failed
    """

    def __init__(self, dictionaries: Sequence, budget_bytes: int = 4 << 30,
                 max_batch: int = 256, streams: int = 4, tune=None, margin: float = 2.0,
                 staging_bytes: int = 256 << 20, copy_threads: int = 8,
                 max_wait_us: int = 200, fail_batch: int = 0):
        self._h = None
        self.dicts = [ac_build(p, sigma=4) for p in dictionaries]
        t = ac_tune()
        if isinstance(tune, ac_tune):
            t = tune
        elif tune:
            t = ac_tune(tune.get("chunk", 0), tune.get("block_threads", 0),
                        tune.get("placement", 0), tune.get("blocks_per_cu", 0),
                        tune.get("chains", 0))
        o = ac_server_opts(int(budget_bytes), int(staging_bytes), int(max_batch), int(streams),
                           int(copy_threads), int(max_wait_us), int(fail_batch), 0,
                           float(margin), t)
        arr = (ctypes.c_void_p * len(self.dicts))(*[d.handle.value for d in self.dicts])
        h = ctypes.c_void_p()
        rc = lib().ac_server_create(arr, len(self.dicts), ctypes.byref(o), ctypes.byref(h))
        if rc != AC_OK:
            raise ACError(rc, "ac_server_create")
        self._h = h
        self._futs: List[ServeFuture] = []
        c = ac_server_counters()
        lib().ac_server_stats(self._h, ctypes.byref(c), None, 0)
        self.budget = c.budget_bytes

    def submit(self, letters: np.ndarray, dict_id: int) -> ServeFuture:
        """Queue a text (uint8 ASCII letters ACGT) for a scan against
        dictionary dict_id.  Returns a future of the uint64 match keys."""
        if not 0 <= dict_id < len(self.dicts):
            raise ValueError("no such dictionary")
        if self._h is None:
            raise RuntimeError("server closed")
        letters = np.ascontiguousarray(letters, dtype=np.uint8)
        ticket = ctypes.c_uint64()
        rc = lib().ac_server_submit(self._h, letters.ctypes.data if len(letters) else None,
                                    len(letters), dict_id, ctypes.byref(ticket))
        if rc == AC_E_HIP:
            raise RuntimeError("server worker failed")
        if rc != AC_OK:
            raise ACError(rc, "ac_server_submit")
        f = ServeFuture(self, ticket.value, letters)
        self._futs.append(f)
        return f

    def request_charge(self, n: int, dict_id: int) -> int:
        """Device bytes a request of n letters for dictionary dict_id would be
        counted against the budget now."""
        b = ctypes.c_uint64()
        rc = lib().ac_server_request_charge(self._h, n, dict_id, ctypes.byref(b))
        if rc != AC_OK:
            raise ACError(rc, "ac_server_request_charge")
        return b.value

    def _drain(self):
        for f in self._futs:
            if not f._done:
                f._fetch(-1)
        self._futs = []

    def close(self) -> ServeStats:
        """Finish every queued request (their futures keep their results)
        and stop the server."""
        if self._h is None:
            raise RuntimeError("server closed")
        self._drain()
        c = ac_server_counters()
        L = lib()
        L.ac_server_stats(self._h, ctypes.byref(c), None, 0)
        lat = np.zeros(max(1, c.requests), dtype=np.float64)
        L.ac_server_stats(self._h, ctypes.byref(c), lat.ctypes.data, c.requests)
        failed = L.ac_server_destroy(self._h)
        self._h = None
        if failed != AC_OK:
            raise RuntimeError("server worker failed")
        return ServeStats(lat[:c.requests].tolist(), c.bases, c.matches, c.batches, c.reruns,
                          c.wall_s, c.peak_bytes, c.overlapped, c.budget_bytes)

    def __del__(self):
        try:
            if self._h is not None:
                self._drain()
                lib().ac_server_destroy(self._h)
                self._h = None
        except Exception:
            pass


def run_poisson(server: Server, texts: Sequence[np.ndarray], dict_of: Sequence[int],
                gaps: Sequence[float], rate: float) -> List[ServeFuture]:
    """Submit texts at Poisson arrival times (gaps are Exp(1) draws scaled
    by 1/rate requests per second), from the calling thread."""
    futs = []
    t0 = time.perf_counter()
    t = 0.0
    for text, d, g in zip(texts, dict_of, gaps):
        t += g / rate
        delay = t0 + t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(server.submit(text, int(d)))
    return futs
