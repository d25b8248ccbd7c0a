"""The paper's pattern-split parallel design on host threads (section IV.A,
second design; Fig. 3), the CPU context baseline: N slices of the pattern
list, one machine and one POSIX thread each, every thread scanning the
whole text.  The union of the slices' matches must be the single machine's
set for any N (the partition invariance that design relies on), and the
per-slice counts must add up to it."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("parts", [1, 2, 3, 8, 16])
def test_split_union_equals_one_machine_dna(parts):
    inst = W.dna_dense(scale=1 / 1024)
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    r = oracle.split_run(inst.patterns, 4, inst.text, parts, collect=True)
    assert int(r["counts"].sum()) == len(want)
    assert np.array_equal(r["keys"], np.sort(want))
    assert r["wall_build_scan_s"] > 0 and r["wall_scan_s"] > 0


@pytest.mark.parametrize("parts", [1, 5, 100])
def test_split_union_equals_one_machine_protein(parts):
    inst = W.protein(scale=1 / 256)
    want = oracle.Machine(inst.patterns, 20).scan_keys(inst.text)
    r = oracle.split_run(inst.patterns, 20, inst.text, parts, collect=True)
    assert np.array_equal(r["keys"], np.sort(want))


def test_split_tiny_corpus_and_count_only():
    for seed in range(200):
        inst = W.tiny(seed, 3)
        want = np.sort(oracle.keys(*oracle.naive_scan(inst.text, inst.patterns)))
        parts = 1 + seed % inst.patterns.count
        r = oracle.split_run(inst.patterns, 3, inst.text, parts, collect=True)
        assert np.array_equal(r["keys"], want), seed
        c = oracle.split_run(inst.patterns, 3, inst.text, parts)
        assert int(c["counts"].sum()) == len(want)


def test_split_rejects_bad_arguments():
    inst = W.dna_small(scale=1 / 64)
    with pytest.raises(oracle.OracleError):
        oracle.split_run(inst.patterns, 4, inst.text, 0)
    with pytest.raises(oracle.OracleError):
        oracle.split_run(inst.patterns, 4, inst.text, inst.patterns.count + 1)
