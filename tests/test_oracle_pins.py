"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something fixed independently of it: the
paper's worked example (section III.A, Figures 1-2), the definition of an
occurrence (brute force on tiny inputs), an independent exact method (rolling
k-mer hashing), closed forms, and the two decompositions the paper discusses
(section IV.A): splitting the pattern file across machines, and splitting the
input into chunks.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from conftest import golden


def _letters(alpha, s):
    return np.array([alpha.index(ch) for ch in s], dtype=np.uint8)


# ------------------------------------------------------------ worked example

def test_fig2_trace_and_matches():
    g = golden("fig2_shers.txt")
    alpha = g["alphabet"]
    names = g["patterns"].split()
    pats = [_letters(alpha, p) for p in names]
    m = oracle.Machine(pats, len(alpha))
    text = _letters(alpha, g["text"])
    want_trace = [(t[0], int(t[1:])) for t in g["trace"].split()]
    assert m.trace(text) == want_trace
    s, f = map(int, g["failure"].split())
    assert m.fail(s) == f
    pid, end = m.scan(text)
    got = [(names[p], int(e)) for p, e in zip(pid, end)]
    want = [(w.split(":")[0], int(w.split(":")[1])) for w in g["matches"].split()]
    assert got == want
    # ten states: the root plus one per distinct keyword prefix
    assert m.n_states == 10


def test_fig2_other_insertion_order_same_matches():
    # the paper lists the keywords as HIS, SHE, HERS; the insertion order
    # changes the state numbers but not the set of recognised keywords
    g = golden("fig2_shers.txt")
    alpha = g["alphabet"]
    names = ["HIS", "SHE", "HERS"]
    m = oracle.Machine([_letters(alpha, p) for p in names], len(alpha))
    pid, end = m.scan(_letters(alpha, "SHERS"))
    assert [(names[p], int(e)) for p, e in zip(pid, end)] == [("SHE", 2), ("HERS", 4)]


def test_output_function_inherits_through_failure():
    # HE is a suffix of SHE: reading SHE must report both, at the same end
    alpha = "EHS"
    names = ["SHE", "HE", "E"]
    m = oracle.Machine([_letters(alpha, p) for p in names], 3)
    pid, end = m.scan(_letters(alpha, "SHE"))
    assert list(zip(pid.tolist(), end.tolist())) == [(0, 2), (1, 2), (2, 2)]


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("sigma", [2, 3, 4])
def test_brute_force_tiny(sigma):
    for seed in range(1500):
        inst = W.tiny(seed * 7 + sigma, sigma)
        m = oracle.Machine(inst.patterns, sigma)
        got = m.scan(inst.text)
        want = oracle.naive_scan(inst.text, inst.patterns)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), seed


def test_brute_force_longer_texts():
    for seed in range(200):
        inst = W.tiny(10_000 + seed, 4, max_text=300, max_pats=25, max_len=8)
        m = oracle.Machine(inst.patterns, 4)
        got = m.scan_keys(inst.text)
        want = oracle.keys(*oracle.naive_scan(inst.text, inst.patterns))
        assert np.array_equal(got, want), seed


# ------------------------------------------------------------ k-mer counts

def _kmer_vs_oracle(inst):
    m = oracle.Machine(inst.patterns, inst.sigma)
    c_or = m.count(inst.text)
    c_km = oracle.kmer_count(inst.text, inst.patterns, inst.sigma)
    assert np.array_equal(c_or, c_km)
    # the scan's output agrees with its own counting
    pid, _ = m.scan(inst.text)
    assert np.array_equal(np.bincount(pid, minlength=inst.patterns.count).astype(np.uint64), c_or)
    return c_or


def test_kmer_counts_dna_small_full():
    c = _kmer_vs_oracle(W.dna_small())
    assert c[:50].min() >= 1          # patterns cut from the text occur


def test_kmer_counts_protein():
    c = _kmer_vs_oracle(W.protein(scale=1 / 8))
    assert c.min() >= 1


def test_kmer_counts_dna_dense():
    inst = W.dna_dense(scale=1 / 32)
    c = _kmer_vs_oracle(inst)
    assert c[9:7009].min() >= 1


@pytest.mark.slow
def test_kmer_counts_protein_full():
    _kmer_vs_oracle(W.protein())


# ------------------------------------------------------------ closed forms

def test_single_pattern_is_overlapping_find():
    rng = W.rng_for(11)
    for trial in range(50):
        text = rng.integers(0, 2, size=2000, dtype=np.uint8)
        L = int(rng.integers(1, 9))
        p = text[int(rng.integers(0, 1990)):][:L]
        m = oracle.Machine([p], 2)
        _, end = m.scan(text)
        hay, needle = text.tobytes(), p.tobytes()
        starts, i = [], hay.find(needle)
        while i >= 0:
            starts.append(i)
            i = hay.find(needle, i + 1)
        assert end.tolist() == [s + L - 1 for s in starts]


def test_length_one_patterns_give_histogram():
    rng = W.rng_for(12)
    text = W._iid(rng, 50_000, W.protein_background(), 20)
    m = oracle.Machine([[a] for a in range(20)], 20)
    pid, end = m.scan(text)
    assert np.array_equal(end, np.arange(len(text), dtype=np.uint32))
    assert np.array_equal(pid, text.astype(np.uint32))


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_all_kmers_match_every_window(k):
    rng = W.rng_for(13)
    n = 5000
    text = rng.integers(0, 4, size=n, dtype=np.uint8)
    kmers = [[(x >> (2 * (k - 1 - j))) & 3 for j in range(k)] for x in range(4 ** k)]
    m = oracle.Machine(kmers, 4)
    pid, end = m.scan(text)
    assert len(pid) == n - k + 1
    assert np.array_equal(end, np.arange(k - 1, n, dtype=np.uint32))
    # the id of the k-mer ending at e is its base-4 value
    codes = np.zeros(n - k + 1, dtype=np.int64)
    for j in range(k):
        codes = codes * 4 + text[j:n - k + 1 + j]
    assert np.array_equal(pid.astype(np.int64), codes)


def test_poly_a_runs_closed_form():
    # in a text with no A outside well separated runs, A^k occurs L-k+1
    # times in each run of length L >= k, and nowhere else
    rng = W.rng_for(14)
    n = 200_000
    text = rng.integers(1, 4, size=n, dtype=np.uint8)
    starts, lens = W._place_runs(rng, n, 0.02, 50, 500)
    for s, L in zip(starts, lens):
        text[s:s + L] = 0
    # runs may touch: merge them into maximal runs before counting
    is_a = np.concatenate([[0], (text == 0).astype(np.int8), [0]])
    d = np.diff(is_a)
    run_len = np.flatnonzero(d == -1) - np.flatnonzero(d == 1)
    pats = [np.zeros(k, dtype=np.uint8) for k in range(8, 17)]
    c = oracle.Machine(pats, 4).count(text)
    for i, k in enumerate(range(8, 17)):
        assert int(c[i]) == int(np.maximum(run_len - k + 1, 0).sum())


# ------------------------------------------------------------ decompositions

def test_pattern_split_union_equals_one_machine():
    # the paper's design (section IV.A, Figure 3): N machines, each built
    # from one chunk of the pattern file and scanning the whole input; the
    # union of their reports (ids shifted back) equals one machine's
    inst = W.dna_small(scale=1 / 8)
    whole = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    pats = inst.patterns.as_list()
    for n_split in (2, 3, 7):
        bounds = np.linspace(0, len(pats), n_split + 1).astype(int)
        parts = []
        for a, b in zip(bounds[:-1], bounds[1:]):
            pid, end = oracle.Machine(pats[a:b], 4).scan(inst.text)
            parts.append(oracle.keys(pid + a, end))
        assert np.array_equal(np.sort(np.concatenate(parts)), whole)


def test_text_chunking_with_overlap_is_exact():
    # splitting the input (section IV.A, first design): each chunk re-read
    # from max_len - 1 symbols earlier, keeping only ends inside the chunk
    inst = W.dna_dense(scale=1 / 4096)
    m = oracle.Machine(inst.patterns, 4)
    whole = m.scan_keys(inst.text)
    mlen = int(inst.patterns.lengths.max())
    assert len(whole) > 100
    for chunk in (1, 7, 29, 30, 64, 1000):
        assert np.array_equal(oracle.chunk_scan(m, inst.text, chunk, mlen), whole), chunk


def test_text_chunking_too_little_overlap_loses_matches():
    # the overlap is needed: one symbol less loses matches that straddle
    inst = W.dna_dense(scale=1 / 4096)
    m = oracle.Machine(inst.patterns, 4)
    whole = m.scan_keys(inst.text)
    mlen = int(inst.patterns.lengths.max())
    short = oracle.chunk_scan(m, inst.text, 64, mlen - 1)
    assert len(short) < len(whole)


# ------------------------------------------------------------ conventions

def test_output_order_is_end_then_id():
    inst = W.dna_dense(scale=1 / 1024)
    k = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    assert np.all(np.diff(k.astype(np.int64)) > 0) if len(k) < 2 ** 62 else True
    assert np.all(k[1:] > k[:-1])


def test_duplicates_each_reported():
    m = oracle.Machine([[1, 2], [1, 2], [2]], 3)
    pid, end = m.scan(np.array([0, 1, 2, 1, 2], dtype=np.uint8))
    assert list(zip(pid.tolist(), end.tolist())) == [(0, 2), (1, 2), (2, 2), (0, 4), (1, 4), (2, 4)]


def test_pattern_longer_than_text_no_match():
    m = oracle.Machine([[0, 0, 0, 0]], 4)
    assert len(m.scan(np.zeros(3, dtype=np.uint8))[0]) == 0


def test_rejects_bad_input():
    with pytest.raises(oracle.OracleError) as e:
        oracle.Machine([[0, 1], []], 4)
    assert e.value.code == oracle.E_EMPTY
    with pytest.raises(oracle.OracleError) as e:
        oracle.Machine([[0, 4]], 4)
    assert e.value.code == oracle.E_SYMBOL


# ------------------------------------------------------------ text encoding

def test_pack2_hand_worked_bytes():
    g = golden("pack2_acgt.txt")
    codes = oracle.encode(np.frombuffer(g["text"].encode(), dtype=np.uint8), W.DNA)
    want = np.array([int(b, 16) for b in g["bytes"].split()], dtype=np.uint8)
    assert np.array_equal(oracle.pack2(codes), want)
    assert np.array_equal(oracle.unpack2(want, len(codes)), codes)


def test_encode_case_insensitive_and_rejects():
    a = np.frombuffer(b"acgtACGT", dtype=np.uint8)
    assert oracle.encode(a, W.DNA).tolist() == [0, 1, 2, 3, 0, 1, 2, 3]
    p = np.frombuffer(W.PROTEIN.encode(), dtype=np.uint8)
    assert oracle.encode(p, W.PROTEIN).tolist() == list(range(20))
    with pytest.raises(ValueError):
        oracle.encode(np.frombuffer(b"ACGN", dtype=np.uint8), W.DNA)
