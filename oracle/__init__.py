"""CPU oracle for the Aho-Corasick scan -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this package.  The product library
(``paper_1403_7294_amd``) never imports it, and it never imports the product
library: the two share no code.  Inputs come from the seeded generators in
``workloads``.

Contents:

* ``Machine``      -- the paper's goto/failure/output automaton and its
                      single-pass scan (section III.A), plain C in
                      ``ac_oracle.c``.
* ``naive_scan``   -- brute force by the definition of an occurrence.
* ``kmer_count``   -- per-pattern counts by rolling k-mer hashing.
* ``encode`` / ``pack2`` / ``unpack2`` -- the text encoding the scan reads:
                      letters -> codes, and DNA codes packed four per byte,
                      least significant bits first.
* ``split_run``    -- the paper's own parallel design on host threads
                      (section IV.A, second design, Fig. 3): N pattern
                      slices, one machine and one POSIX thread each, every
                      thread reading the whole text; plain C in
                      ``ac_split.c`` over the same machine.  The CPU context
                      baseline, timed build + scan and scan only.
* ``chunk_scan``   -- the text-chunking rule (each chunk re-read from
                      ``max(0, start - (m_max - 1))``, reporting only ends
                      inside the chunk) applied to the oracle's scan.

Results are returned as ``(pid, end)`` uint32 arrays in (end, pid) order, or
as uint64 keys ``end << 32 | pid`` (sorted ascending = (end, pid) order).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["ac_oracle.c", "naive.c", "ac_split.c"]
_lib = None

OK, E_INVALID, E_EMPTY, E_SYMBOL, E_TOO_LARGE, E_NOMEM = 0, -1, -2, -3, -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle's C sources into liboracle.so (gcc, -O2)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                    "-pthread", "-o", tmp] + srcs, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = _open(_LIB_PATH)
    return _lib


def _open(path: str):
    """Load a compiled oracle library and declare its signatures."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    u32, u64, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
    lib.oracle_build.argtypes = [P, P, u32, u32, ctypes.POINTER(P)]
    lib.oracle_build.restype = ctypes.c_int
    lib.oracle_free.argtypes = [P]
    lib.oracle_free.restype = None
    lib.oracle_scan.argtypes = [P, P, u64, P, P, u64]
    lib.oracle_scan.restype = i64
    lib.oracle_count.argtypes = [P, P, u64, P, u32]
    lib.oracle_count.restype = ctypes.c_int
    lib.oracle_trace.argtypes = [P, P, u64, P, P, u64]
    lib.oracle_trace.restype = i64
    lib.oracle_num_states.argtypes = [P]
    lib.oracle_num_states.restype = u32
    lib.oracle_goto.argtypes = [P, u32, u32]
    lib.oracle_goto.restype = ctypes.c_int32
    lib.oracle_fail.argtypes = [P, u32]
    lib.oracle_fail.restype = ctypes.c_int32
    lib.oracle_depth.argtypes = [P, u32]
    lib.oracle_depth.restype = u32
    lib.oracle_output.argtypes = [P, u32, P, u64]
    lib.oracle_output.restype = i64
    lib.naive_scan.argtypes = [P, u64, P, P, u32, P, P, u64]
    lib.naive_scan.restype = i64
    lib.kmer_count.argtypes = [P, u64, P, P, u32, u32, P]
    lib.kmer_count.restype = ctypes.c_int
    if hasattr(lib, "split_run"):  # absent from copies built without ac_split.c
        d = ctypes.POINTER(ctypes.c_double)
        lib.split_run.argtypes = [P, P, u32, u32, P, u64, u32, P, P, u64, P, d, d, P, P]
        lib.split_run.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _csr(patterns) -> Tuple[np.ndarray, np.ndarray]:
    if hasattr(patterns, "symbols"):
        sym, off = patterns.symbols, patterns.offsets
    else:
        lens = [len(p) for p in patterns]
        off = np.zeros(len(lens) + 1, dtype=np.uint64)
        np.cumsum(lens, out=off[1:])
        sym = (np.concatenate([np.asarray(p, dtype=np.uint8) for p in patterns])
               if off[-1] else np.zeros(1, dtype=np.uint8))
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    if sym.size == 0:
        sym = np.zeros(1, dtype=np.uint8)
    return sym, np.ascontiguousarray(off, dtype=np.uint64)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


def keys(pid: np.ndarray, end: np.ndarray) -> np.ndarray:
    """uint64 keys end << 32 | pid (ascending order = (end, pid) order)."""
    return (end.astype(np.uint64) << np.uint64(32)) | pid.astype(np.uint64)


class Machine:
    """The paper's goto/failure/output machine over codes 0..sigma-1."""

    def __init__(self, patterns, sigma: int):
        lib = _load()
        sym, off = _csr(patterns)
        self.n_patterns = len(off) - 1
        self.sigma = sigma
        h = ctypes.c_void_p()
        rc = lib.oracle_build(_ptr(sym), _ptr(off), self.n_patterns, sigma, ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc)
        self._h = h
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.oracle_free(h)
            self._h = None

    def scan(self, text: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        text = np.ascontiguousarray(text, dtype=np.uint8)
        cap = max(16, len(text))
        while True:
            pid = np.empty(cap, dtype=np.uint32)
            end = np.empty(cap, dtype=np.uint32)
            tot = self._lib.oracle_scan(self._h, _ptr(text), len(text), _ptr(pid), _ptr(end), cap)
            if tot < 0:
                raise OracleError(int(tot))
            if tot <= cap:
                return pid[:tot], end[:tot]
            cap = int(tot)

    def scan_keys(self, text: np.ndarray) -> np.ndarray:
        return keys(*self.scan(text))

    def count(self, text: np.ndarray) -> np.ndarray:
        text = np.ascontiguousarray(text, dtype=np.uint8)
        c = np.zeros(self.n_patterns, dtype=np.uint64)
        rc = self._lib.oracle_count(self._h, _ptr(text), len(text), _ptr(c), self.n_patterns)
        if rc != OK:
            raise OracleError(rc)
        return c

    def trace(self, text: np.ndarray):
        text = np.ascontiguousarray(text, dtype=np.uint8)
        cap = 4 * len(text) + 16
        st = np.empty(cap, dtype=np.int32)
        kd = np.empty(cap, dtype=np.uint8)
        k = self._lib.oracle_trace(self._h, _ptr(text), len(text), _ptr(st), _ptr(kd), cap)
        if k < 0:
            raise OracleError(int(k))
        assert k <= cap
        return [(chr(kd[i]), int(st[i])) for i in range(k)]

    @property
    def n_states(self) -> int:
        return int(self._lib.oracle_num_states(self._h))

    def goto(self, s: int, a: int) -> int:
        return int(self._lib.oracle_goto(self._h, s, a))

    def fail(self, s: int) -> int:
        return int(self._lib.oracle_fail(self._h, s))

    def depth(self, s: int) -> int:
        return int(self._lib.oracle_depth(self._h, s))

    def output(self, s: int) -> np.ndarray:
        n = self._lib.oracle_output(self._h, s, ctypes.c_void_p(0), 0)
        ids = np.empty(max(1, n), dtype=np.uint32)
        self._lib.oracle_output(self._h, s, _ptr(ids), n)
        return ids[:n]


def naive_scan(text: np.ndarray, patterns) -> Tuple[np.ndarray, np.ndarray]:
    lib = _load()
    text = np.ascontiguousarray(text, dtype=np.uint8)
    sym, off = _csr(patterns)
    npat = len(off) - 1
    cap = max(16, len(text) * max(1, npat))
    pid = np.empty(cap, dtype=np.uint32)
    end = np.empty(cap, dtype=np.uint32)
    tot = lib.naive_scan(_ptr(text) if len(text) else ctypes.c_void_p(0), len(text),
                         _ptr(sym), _ptr(off), npat, _ptr(pid), _ptr(end), cap)
    assert 0 <= tot <= cap
    return pid[:tot], end[:tot]


def kmer_count(text: np.ndarray, patterns, sigma: int) -> np.ndarray:
    lib = _load()
    text = np.ascontiguousarray(text, dtype=np.uint8)
    sym, off = _csr(patterns)
    npat = len(off) - 1
    c = np.zeros(npat, dtype=np.uint64)
    rc = lib.kmer_count(_ptr(text) if len(text) else ctypes.c_void_p(0), len(text),
                        _ptr(sym), _ptr(off), npat, sigma, _ptr(c))
    if rc != 0:
        raise OracleError(rc)
    return c


def split_run(patterns, sigma: int, text: np.ndarray, parts: int, collect: bool = False) -> dict:
    """The paper's second parallel design with ``parts`` POSIX threads: slice
    t of the pattern list (consecutive patterns, sizes within one) gets its
    own machine and thread, and every thread scans the whole text.  Returns
    the per-slice match counts, the wall time of one run that builds and
    scans (what the paper timed) and of a second run of the same machines
    that only scans, the per-thread build and scan times of the first run,
    and, with ``collect``, the union of all slices' matches as sorted uint64
    keys (global pattern ids)."""
    lib = _load()
    text = np.ascontiguousarray(text, dtype=np.uint8)
    sym, off = _csr(patterns)
    npat = len(off) - 1
    counts = np.zeros(parts, dtype=np.uint64)
    bs = np.zeros(parts, dtype=np.float64)
    ss = np.zeros(parts, dtype=np.float64)
    w1, w2 = ctypes.c_double(), ctypes.c_double()
    cap = 0
    pid = end = np.zeros(1, dtype=np.uint32)
    while True:
        rc = lib.split_run(_ptr(sym), _ptr(off), npat, sigma,
                           _ptr(text) if len(text) else ctypes.c_void_p(0), len(text), parts,
                           _ptr(pid) if cap else ctypes.c_void_p(0),
                           _ptr(end) if cap else ctypes.c_void_p(0), cap, _ptr(counts),
                           ctypes.byref(w1), ctypes.byref(w2), _ptr(bs), _ptr(ss))
        if rc != OK:
            raise OracleError(rc)
        need = int(counts.max()) if parts else 0
        if not collect or need <= cap:
            break
        cap = need
        pid = np.empty(parts * cap, dtype=np.uint32)
        end = np.empty(parts * cap, dtype=np.uint32)
    res = {"parts": parts, "counts": counts, "wall_build_scan_s": w1.value,
           "wall_scan_s": w2.value, "build_s": bs, "scan_s": ss}
    if collect:
        sel = np.concatenate([np.arange(t * cap, t * cap + int(counts[t])) for t in range(parts)]
                             ) if cap else np.zeros(0, dtype=np.int64)
        res["keys"] = np.sort(keys(pid[sel], end[sel]))
    return res


# ------------------------------------------------------------- text encoding

def encode(ascii_text: np.ndarray, alphabet: str) -> np.ndarray:
    """Letters -> codes by position in ``alphabet`` (case-insensitive).

    Raises ValueError on a letter outside the alphabet."""
    lut = np.full(256, 255, dtype=np.uint8)
    for code, letter in enumerate(alphabet):
        lut[ord(letter.upper())] = code
        lut[ord(letter.lower())] = code
    codes = lut[np.asarray(ascii_text, dtype=np.uint8)]
    if codes.size and codes.max() == 255:
        raise ValueError("letter outside the alphabet")
    return codes


def pack2(codes: np.ndarray) -> np.ndarray:
    """DNA codes (0..3) -> bytes, four bases per byte: base i sits in byte
    i // 4 at bits 2*(i % 4) and 2*(i % 4) + 1; unused high bits of the last
    byte are zero."""
    codes = np.asarray(codes, dtype=np.uint8)
    if codes.size and codes.max() > 3:
        raise ValueError("not a 2-bit code")
    n = len(codes)
    padded = np.zeros((n + 3) // 4 * 4, dtype=np.uint8)
    padded[:n] = codes
    q = padded.reshape(-1, 4)
    return (q[:, 0] | (q[:, 1] << 2) | (q[:, 2] << 4) | (q[:, 3] << 6)).astype(np.uint8)


def unpack2(packed: np.ndarray, n: int) -> np.ndarray:
    packed = np.asarray(packed, dtype=np.uint8)
    out = np.empty((len(packed), 4), dtype=np.uint8)
    for j in range(4):
        out[:, j] = (packed >> (2 * j)) & 3
    return out.reshape(-1)[:n]


# --------------------------------------------------------- chunking rule

def chunk_scan(machine: Machine, text: np.ndarray, chunk: int, max_len: int) -> np.ndarray:
    """Keys of the matches found by scanning each chunk [jC, (j+1)C) from
    max(0, jC - (max_len - 1)) with a fresh machine state and keeping only
    ends inside the chunk.  Equals ``machine.scan_keys(text)`` when the
    overlap is at least max_len - 1 (this is what the tests check)."""
    n = len(text)
    parts = []
    for j0 in range(0, n, chunk):
        s = max(0, j0 - (max_len - 1))
        e = min(n, j0 + chunk)
        pid, end = machine.scan(text[s:e])
        end = end.astype(np.int64) + s
        keep = end >= j0
        parts.append(keys(pid[keep], end[keep].astype(np.uint32)))
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)


def batch_scan(instances: Sequence) -> list:
    """Keys for each (text, patterns, sigma) instance, scanned one by one."""
    return [Machine(i.patterns, i.sigma).scan_keys(i.text) for i in instances]
