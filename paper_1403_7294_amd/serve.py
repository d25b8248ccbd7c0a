"""Continuous-batching server for Aho-Corasick scans on one GPU.

Requests (a text as letters, and the index of one of the server's
device-resident dictionaries) arrive at any time through ``submit``.  A
worker thread admits waiting requests while the device-memory budget and the
batch slots allow, packs them into one batch, and runs the batch on one of
several streams: host-to-device copy of the letters, ``ac_encode`` into
2-bit text, ``ac_scan_batch`` over all requests of the batch, copy of the
matches back.  Requests that arrive while batches are running are admitted
into the next batch at once, so their work overlaps the batches already on
the GPU; memory is released, and further requests admitted, as batches
complete.  Each request's future resolves to its matches (uint64 keys
``end << 32 | pattern_id`` in (end, id) order) - the same result the request
would get from a scan alone.

Output space is reserved per request from a running estimate of the
dictionary's matches per base; a request whose matches overflow its
reservation is scanned again, alone, with an exact-size buffer.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import threading
import time
from typing import List, Optional, Sequence

import numpy as np

from . import (AC_ALPHA_DNA, AC_TEXT_2BIT, ac_build, ac_encode, ac_scan, ac_scan_batch,
               match_keys)


@dataclasses.dataclass
class _Request:
    rid: int
    dict_id: int
    letters: np.ndarray
    arrival: float
    future: concurrent.futures.Future
    capacity: int = 0
    nbytes: int = 0
    done: float = 0.0


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
                "peak_device_bytes": self.peak_bytes}


class Server:
    """Serve scans of DNA texts against dictionaries kept on the GPU.

    dictionaries  list of pattern sets (code lists or CSR objects), DNA codes
    budget_bytes  device memory the server may hold for requests at once
    max_batch     requests per batch
    streams       batches in flight at once (>= 2 to overlap)
    """

    def __init__(self, dictionaries: Sequence, budget_bytes: int = 4 << 30,
                 max_batch: int = 64, streams: int = 2, tune=None,
                 margin: float = 2.0):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.dicts = [ac_build(p, sigma=4) for p in dictionaries]
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(max(2, streams))]
        self.tune = tune
        self.margin = margin
        # matches per base, per dictionary (running estimate)
        self.rate = [1e-3] * len(self.dicts)
        self._q: collections.deque = collections.deque()
        self._cv = threading.Condition()
        self._closing = False
        self._next_id = 0
        self._used = 0
        self._peak = 0
        self._lat: List[float] = []
        self._bases = 0
        self._matches = 0
        self._batches = 0
        self._reruns = 0
        self._overlapped = 0
        self._t0: Optional[float] = None
        self._t_last = 0.0
        self._err: Optional[BaseException] = None
        self._worker = threading.Thread(target=self._run, name="ac-serve", daemon=True)
        self._worker.start()

    # ------------------------------------------------------------ client API

    def submit(self, letters: np.ndarray, dict_id: int) -> concurrent.futures.Future:
        """Queue a text (uint8 ASCII letters ACGT) for a scan against
        dictionary dict_id.  Returns a future of the uint64 match keys."""
        if not 0 <= dict_id < len(self.dicts):
            raise ValueError("no such dictionary")
        f: concurrent.futures.Future = concurrent.futures.Future()
        letters = np.ascontiguousarray(letters, dtype=np.uint8)
        with self._cv:
            if self._closing:
                raise RuntimeError("server closed")
            r = _Request(self._next_id, dict_id, letters, time.perf_counter(), f)
            self._next_id += 1
            self._size(r)
            if r.nbytes > self.budget:
                f.set_exception(MemoryError("request larger than the server's memory budget"))
                return f
            if self._t0 is None:
                self._t0 = r.arrival
            self._q.append(r)
            self._cv.notify()
        return f

    def close(self) -> ServeStats:
        """Finish every queued request and stop the worker."""
        with self._cv:
            self._closing = True
            self._cv.notify()
        self._worker.join()
        if self._err is not None:
            raise self._err
        wall = (self._t_last - self._t0) if self._t0 is not None else 0.0
        return ServeStats(self._lat, self._bases, self._matches, self._batches, self._reruns,
                          wall, self._peak, self._overlapped)

    # ------------------------------------------------------------ internals

    def _size(self, r: _Request):
        n = len(r.letters)
        est = int(self.rate[r.dict_id] * n * self.margin) + 64
        r.capacity = est
        # letters (padded) + packed text + matches + count
        r.nbytes = _pad16(n) + _pad16(n) // 4 + 8 * est + 8

    def _take(self, n_inflight: int) -> List[_Request]:
        """Admit queued requests in arrival order while memory and slots allow
        (caller holds the lock)."""
        batch: List[_Request] = []
        if n_inflight >= len(self.streams):
            return batch
        while (self._q and len(batch) < self.max_batch and
               self._used + self._q[0].nbytes <= self.budget):
            r = self._q.popleft()
            self._used += r.nbytes
            batch.append(r)
        self._peak = max(self._peak, self._used)
        return batch

    def _run(self):
        try:
            inflight: collections.deque = collections.deque()
            k = 0
            while True:
                while inflight and inflight[0]["event"].query():
                    self._finish(inflight.popleft())
                with self._cv:
                    batch = self._take(len(inflight))
                    if not batch:
                        if not inflight:
                            if self._closing and not self._q:
                                return
                            self._cv.wait(timeout=0.05)
                            continue
                        blocked = bool(self._q)  # slots or memory exhausted
                        if not blocked:
                            # wait for an arrival, then look at the GPU again
                            self._cv.wait(timeout=2e-4)
                            continue
                if not batch:
                    self._finish(inflight.popleft())  # blocks on the oldest batch
                    continue
                st = self.streams[k % len(self.streams)]
                k += 1
                if inflight:
                    self._overlapped += 1
                inflight.append(self._launch(batch, st))
        except BaseException as e:  # surface worker failures to close()
            self._err = e
            with self._cv:
                for r in self._q:
                    r.future.set_exception(e)
                self._q.clear()

    def _launch(self, batch: List[_Request], st) -> dict:
        torch = self.torch
        offs = np.zeros(len(batch) + 1, dtype=np.int64)
        for i, r in enumerate(batch):
            offs[i + 1] = offs[i] + _pad16(len(r.letters))
        host = torch.empty(int(offs[-1]), dtype=torch.uint8, pin_memory=True)
        hv = host.numpy()
        hv[:] = ord("A")
        for i, r in enumerate(batch):
            hv[offs[i]:offs[i] + len(r.letters)] = r.letters
        caps = np.array([r.capacity for r in batch], dtype=np.int64)
        moff = np.zeros(len(batch) + 1, dtype=np.int64)
        np.cumsum(caps, out=moff[1:])
        with torch.cuda.stream(st):
            letters = torch.empty(int(offs[-1]), dtype=torch.uint8, device=self.dev)
            letters.copy_(host, non_blocking=True)
            packed = torch.empty(int(offs[-1]) // 4, dtype=torch.uint8, device=self.dev)
            bad = torch.zeros(1, dtype=torch.int64, device=self.dev)
            ac_encode(letters, AC_ALPHA_DNA, AC_TEXT_2BIT, packed, bad, stream=st)
            out = torch.empty((int(moff[-1]), 2), dtype=torch.int32, device=self.dev)
            counts = torch.zeros(len(batch), dtype=torch.int64, device=self.dev)
            items = []
            for i, r in enumerate(batch):
                t = packed[offs[i] // 4:offs[i + 1] // 4]
                items.append((self.dicts[r.dict_id], t, len(r.letters), AC_TEXT_2BIT,
                              out[moff[i]:moff[i + 1]], int(caps[i]), counts[i:i + 1]))
            ac_scan_batch(items, tune=self.tune, stream=st)
            counts_host = torch.empty(len(batch) + 1, dtype=torch.int64, pin_memory=True)
            counts_host[:len(batch)].copy_(counts, non_blocking=True)
            counts_host[len(batch):].copy_(bad, non_blocking=True)
            # the reserved output comes back in one copy; the host reads what
            # each request filled once the batch is done
            out_host = torch.empty(out.shape, dtype=torch.int32, pin_memory=True)
            out_host.copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        return {"batch": batch, "stream": st, "event": ev, "out": out, "moff": moff,
                "counts": counts_host, "out_host": out_host, "packed": packed, "offs": offs, "keep": (host, letters)}

    def _finish(self, b: dict):
        torch = self.torch
        b["event"].synchronize()
        counts = b["counts"].numpy()
        batch: List[_Request] = b["batch"]
        st = b["stream"]
        results: list = []
        invalid = counts[len(batch)] != 0
        with torch.cuda.stream(st):
            for i, r in enumerate(batch):
                c = int(counts[i])
                if invalid and not _dna_letters(r.letters):
                    # the encoder counted letters outside ACGTacgt in this batch
                    results.append(ValueError("request text has letters outside ACGTacgt"))
                elif c <= r.capacity:
                    m = b["out_host"][b["moff"][i]:b["moff"][i] + c]
                    results.append(match_keys(m))
                else:
                    # overflow: scan this request again, alone, exactly sized
                    self._reruns += 1
                    t = b["packed"][b["offs"][i] // 4:b["offs"][i + 1] // 4]
                    o = torch.empty((c, 2), dtype=torch.int32, device=self.dev)
                    cnt = torch.zeros(1, dtype=torch.int64, device=self.dev)
                    ac_scan(self.dicts[r.dict_id], t, len(r.letters), AC_TEXT_2BIT, o, c, cnt,
                            tune=self.tune, stream=st)
                    st.synchronize()
                    results.append(match_keys(o))
        now = time.perf_counter()
        with self._cv:
            for r, res in zip(batch, results):
                self._used -= r.nbytes
                if isinstance(res, Exception):
                    continue
                n = len(r.letters)
                if n:
                    self.rate[r.dict_id] = 0.8 * self.rate[r.dict_id] + 0.2 * (len(res) / n)
                self._lat.append(now - r.arrival)
                self._bases += n
                self._matches += len(res)
            self._batches += 1
            self._t_last = now
            self._cv.notify()
        for r, res in zip(batch, results):
            if isinstance(res, Exception):
                r.future.set_exception(res)
            else:
                r.future.set_result(res)


def _pad16(n: int) -> int:
    return (n + 15) // 16 * 16


_DNA_OK = np.zeros(256, dtype=bool)
_DNA_OK[np.frombuffer(b"ACGTacgt", dtype=np.uint8)] = True


def _dna_letters(letters: np.ndarray) -> bool:
    return bool(_DNA_OK[letters].all())


def run_poisson(server: Server, texts: Sequence[np.ndarray], dict_of: Sequence[int],
                gaps: Sequence[float], rate: float) -> List[concurrent.futures.Future]:
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
