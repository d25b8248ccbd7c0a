"""Seeded synthetic inputs for the Aho-Corasick scan (DNA and protein).

This module draws random texts and pattern sets and nothing else: it holds
none of the matching arithmetic, and both the CPU oracle (``oracle/``) and the
HIP library (``paper_1403_7294_amd``) consume what it returns.  Every draw
comes from ``numpy.random.Generator(PCG64(seed))``.

Symbols are small integer codes; the letter order of each alphabet fixes the
code of each letter (DNA ``ACGT`` -> 0..3, protein ``ACDEFGHIKLMNPQRSTVWY`` ->
0..19).  The paper (section IV.B) reads patterns one per line and the text
from a file; here patterns are a CSR pair (``symbols``, ``offsets``) with
pattern ``i`` = ``symbols[offsets[i]:offsets[i+1]]``, ids in input order.

The five workloads follow the configurations the scan is measured on:

* ``dna_small``      1,048,576 uniform DNA bases, 100 patterns of 8-16
                     (50 cut from the text, 50 random).
* ``dna_dense``      268,435,456 DNA bases, GC 0.4, 1 % of the text in poly-A
                     runs of 50-500; 10,000 patterns: A^8..A^16, 7,000 cut
                     (10-30), 2,991 random from the background (10-30).
* ``protein``        67,108,864 residues with a skewed background
                     (max 10 %, min 1.3 %), 5,000 cut patterns of 5-12.
* ``batch``          512 DNA instances, text lengths log-uniform 4 Ki-4 Mi,
                     pattern counts log-uniform 10-2,000, lengths 8-24.
* ``serve``          8 DNA dictionaries of 1,000-50,000 patterns (10-30) and a
                     Poisson request stream, lengths log-uniform 1 K-1 M.

Every generator takes a ``scale`` in (0, 1] that shrinks the text (and, for
``batch``/``serve``, the instance sizes) while keeping the recipe, so tests
can run the same distributions at sizes the oracle finishes in seconds.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence

import numpy as np

DNA = "ACGT"
PROTEIN = "ACDEFGHIKLMNPQRSTVWY"


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class PatternSet:
    """CSR pattern list: pattern i = symbols[offsets[i]:offsets[i+1]]."""

    symbols: np.ndarray  # uint8 codes
    offsets: np.ndarray  # uint64, len = count + 1

    @property
    def count(self) -> int:
        return len(self.offsets) - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def pattern(self, i: int) -> np.ndarray:
        return self.symbols[int(self.offsets[i]):int(self.offsets[i + 1])]

    def as_list(self) -> List[np.ndarray]:
        return [self.pattern(i) for i in range(self.count)]

    @staticmethod
    def from_list(pats: Sequence[Sequence[int]]) -> "PatternSet":
        lens = np.array([len(p) for p in pats], dtype=np.uint64)
        off = np.zeros(len(pats) + 1, dtype=np.uint64)
        np.cumsum(lens, out=off[1:])
        sym = (np.concatenate([np.asarray(p, dtype=np.uint8) for p in pats])
               if len(pats) and off[-1] > 0 else np.zeros(0, dtype=np.uint8))
        return PatternSet(sym.astype(np.uint8), off)


@dataclasses.dataclass
class Instance:
    """One (text, dictionary) pair."""

    text: np.ndarray  # uint8 codes, one symbol per byte
    patterns: PatternSet
    sigma: int
    alphabet: str
    name: str = ""

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(self.text.tobytes())
        h.update(self.patterns.symbols.tobytes())
        h.update(self.patterns.offsets.tobytes())
        return h.hexdigest()


def to_ascii(codes: np.ndarray, alphabet: str) -> np.ndarray:
    """Letters for the given codes (uint8 ASCII array)."""
    table = np.frombuffer(alphabet.encode("ascii"), dtype=np.uint8)
    return table[codes]


def _iid(rng: np.random.Generator, n: int, probs: Optional[np.ndarray], sigma: int) -> np.ndarray:
    if probs is None:
        return rng.integers(0, sigma, size=n, dtype=np.uint8)
    cdf = np.cumsum(probs)
    cdf[-1] = 1.0
    u = rng.random(n)
    return np.searchsorted(cdf, u, side="right").astype(np.uint8)


def _cut(rng: np.random.Generator, text: np.ndarray, lengths: np.ndarray) -> List[np.ndarray]:
    out = []
    n = len(text)
    for L in lengths:
        L = int(min(L, n))
        o = int(rng.integers(0, n - L + 1))
        out.append(text[o:o + L].copy())
    return out


def _random_pats(rng, lengths, probs, sigma) -> List[np.ndarray]:
    return [_iid(rng, int(L), probs, sigma) for L in lengths]


# ---------------------------------------------------------------- configs

def dna_small(seed: int = 1, scale: float = 1.0) -> Instance:
    rng = rng_for(seed)
    n = max(64, int(round(1_048_576 * scale)))
    text = rng.integers(0, 4, size=n, dtype=np.uint8)
    lens = rng.integers(8, 17, size=100)
    pats = _cut(rng, text, lens[:50]) + _random_pats(rng, lens[50:], None, 4)
    return Instance(text, PatternSet.from_list(pats), 4, DNA, "dna_small")


def _place_runs(rng, n: int, frac: float, lo: int, hi: int):
    """Non-overlapping run placement: returns (starts, lengths)."""
    target = int(math.ceil(frac * n))
    lens = []
    tot = 0
    while tot < target:
        L = int(rng.integers(lo, hi + 1))
        lens.append(L)
        tot += L
    lens = np.array(lens, dtype=np.int64)
    free = n - tot
    if free < 0:
        raise ValueError("runs do not fit")
    cuts = np.sort(rng.integers(0, free + 1, size=len(lens)))
    starts = cuts + np.concatenate([[0], np.cumsum(lens)[:-1]])
    return starts.astype(np.int64), lens


DNA_DENSE_BG = np.array([0.3, 0.2, 0.2, 0.3])  # A C G T, GC = 0.4


def dna_dense(seed: int = 2, scale: float = 1.0) -> Instance:
    rng = rng_for(seed)
    n = max(4096, int(round(268_435_456 * scale)))
    # background: 10 equiprobable draws mapped A,A,A,C,C,G,G,T,T,T gives
    # exactly P(A)=P(T)=0.3, P(C)=P(G)=0.2
    lut = np.array([0, 0, 0, 1, 1, 2, 2, 3, 3, 3], dtype=np.uint8)
    text = lut[rng.integers(0, 10, size=n, dtype=np.uint8)]
    starts, lens = _place_runs(rng, n, 0.01, 50, 500)
    for s, L in zip(starts, lens):
        text[s:s + L] = 0
    pats = [np.zeros(k, dtype=np.uint8) for k in range(8, 17)]
    cut_lens = rng.integers(10, 31, size=7000)
    pats += _cut(rng, text, cut_lens)
    rnd_lens = rng.integers(10, 31, size=2991)
    pats += _random_pats(rng, rnd_lens, DNA_DENSE_BG, 4)
    inst = Instance(text, PatternSet.from_list(pats), 4, DNA, "dna_dense")
    inst.runs = (starts, lens)  # type: ignore[attr-defined]
    return inst


def protein_background() -> np.ndarray:
    f = np.concatenate([[0.100], np.linspace(0.085, 0.01356, 18), [0.013]])
    return f / f.sum()


def protein(seed: int = 3, scale: float = 1.0) -> Instance:
    rng = rng_for(seed)
    n = max(4096, int(round(67_108_864 * scale)))
    text = _iid(rng, n, protein_background(), 20)
    lens = rng.integers(5, 13, size=5000)
    pats = _cut(rng, text, lens)
    return Instance(text, PatternSet.from_list(pats), 20, PROTEIN, "protein")


def _log_uniform_int(rng, lo, hi, size):
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)


def batch(seed: int = 4, scale: float = 1.0, count: int = 512) -> List[Instance]:
    """Independent DNA instances of very uneven size."""
    rng = rng_for(seed)
    tl = _log_uniform_int(rng, 4096, 4 * 1024 * 1024, count)
    tl = np.maximum(64, np.round(tl * scale).astype(np.int64))
    pc = _log_uniform_int(rng, 10, 2000, count)
    out = []
    for i in range(count):
        text = rng.integers(0, 4, size=int(tl[i]), dtype=np.uint8)
        lens = rng.integers(8, 25, size=int(pc[i]))
        h = len(lens) // 2
        pats = _cut(rng, text, lens[:h]) + _random_pats(rng, lens[h:], None, 4)
        out.append(Instance(text, PatternSet.from_list(pats), 4, DNA, f"batch{i}"))
    return out


@dataclasses.dataclass
class ServeWorkload:
    dictionaries: List[PatternSet]
    texts: List[np.ndarray]      # request texts (uint8 DNA codes)
    dict_of: np.ndarray          # dictionary index of each request
    gaps: np.ndarray             # inter-arrival gaps in units of 1/rate (Exp(1))


def serve(seed: int = 5, scale: float = 1.0, requests: int = 10_000,
          dict_scale: float = 1.0) -> ServeWorkload:
    rng = rng_for(seed)
    counts = np.round(np.geomspace(1000, 50000, 8) * dict_scale).astype(np.int64)
    counts = np.maximum(counts, 4)
    dicts = []
    for c in counts:
        lens = rng.integers(10, 31, size=int(c))
        dicts.append(PatternSet.from_list(_random_pats(rng, lens, None, 4)))
    lens = _log_uniform_int(rng, 1000, 1_000_000, requests)
    lens = np.maximum(16, np.round(lens * scale).astype(np.int64))
    texts = [rng.integers(0, 4, size=int(L), dtype=np.uint8) for L in lens]
    dict_of = rng.integers(0, 8, size=requests)
    gaps = rng.exponential(1.0, size=requests)
    return ServeWorkload(dicts, texts, dict_of, gaps)


def tiny(seed: int, sigma: int, max_text: int = 12, max_pats: int = 6,
         max_len: int = 5) -> Instance:
    """Tiny random instance with nested/duplicated patterns, for brute force."""
    rng = rng_for(seed)
    n = int(rng.integers(0, max_text + 1))
    text = rng.integers(0, sigma, size=n, dtype=np.uint8)
    k = int(rng.integers(1, max_pats + 1))
    pats: List[np.ndarray] = []
    for _ in range(k):
        r = rng.random()
        if pats and r < 0.2:
            pats.append(pats[int(rng.integers(0, len(pats)))].copy())  # duplicate
        elif pats and r < 0.4:
            p = pats[int(rng.integers(0, len(pats)))]
            a = int(rng.integers(0, len(p)))
            b = int(rng.integers(a + 1, len(p) + 1))
            pats.append(p[a:b].copy())  # nested substring
        elif n and r < 0.7:
            L = int(rng.integers(1, max_len + 1))
            pats.extend(_cut(rng, text, np.array([L])))
        else:
            L = int(rng.integers(1, max_len + 1))
            pats.append(rng.integers(0, sigma, size=L, dtype=np.uint8))
    return Instance(text, PatternSet.from_list(pats), sigma, "", f"tiny{seed}")


CONFIGS = {
    "dna_small": dna_small,
    "dna_dense": dna_dense,
    "protein": protein,
}
