"""GPU parity of the 2-bit hybrid count walk (hot rows in LDS as 16-bit ids,
the rest read from the count table that carries each target's output-set
size) and of the dense emit's run writer, against the CPU oracle.

The cases aim at the walk's special paths: few hot rows (most lookups go
to the global table, and every transition into an output state is an
escape from a hot row), texts whose last word is partial, output sets of
up to 16, 64, 128 and more ids (the dense emit's scalar, one-shuffle,
two-shuffle and per-position paths), sets beyond the count table's 8-bit
size field (the scan falls back to the general walk), and capacities that
cut a dense run."""
import sys

import numpy as np
import pytest

import oracle
import paper_1403_7294_amd as ac
import workloads as W
from gpu_helpers import device_text, gpu_keys, torch_cuda

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _instance(seed, n, dups):
    """DNA text with poly-A runs; A^k patterns, cuts of the text, random
    patterns and `dups` copies of A^12 (large output sets in the runs)."""
    rng = W.rng_for(seed)
    text = rng.integers(0, 4, size=n, dtype=np.uint8)
    for start in range(7, max(8, n - 40), 2500):
        text[start:start + int(rng.integers(20, 600))] = 0
    pats = [np.zeros(k, np.uint8) for k in range(3, 17)]
    pats += [np.zeros(12, np.uint8)] * dups
    if n > 40:
        pats += W._cut(rng, text, rng.integers(6, 20, size=150))
    pats += [rng.integers(0, 4, size=int(L), dtype=np.uint8) for L in rng.integers(6, 20, size=80)]
    return W.Instance(text, W.PatternSet.from_list(pats), 4, W.DNA, f"hybrid_{seed}")


def _check(inst, d, tune, capacity=None):
    t = device_text(inst, ac.AC_TEXT_2BIT)
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    got, total = gpu_keys(d, t, len(inst.text), ac.AC_TEXT_2BIT, tune=tune, capacity=capacity)
    assert total == len(want)
    cap = len(want) if capacity is None else min(capacity, len(want))
    assert np.array_equal(got[:cap], want[:cap])
    return len(want)


@pytest.mark.parametrize("n", [5, 16, 65, 64 * 1000 + 17, 100_003])
@pytest.mark.parametrize("hot", [0, 20, 300])
def test_hybrid_walk_tails_and_cold_rows(n, hot):
    inst = _instance(11 + n, n, dups=0)
    d = ac.ac_build(inst.patterns, sigma=4, hot_states=hot)
    for tune in ({"placement": ac.AC_PLACE_HYBRID},
                 {"placement": ac.AC_PLACE_HYBRID, "chains": 1, "chunk": 64},
                 {"placement": ac.AC_PLACE_HYBRID, "chains": 4, "chunk": 256,
                  "block_threads": 256}):
        _say("n", n, "hot rows", hot, "tune", tune)
        _check(inst, d, tune)


@pytest.mark.parametrize("dups", [10, 40, 90, 150, 300])
def test_hybrid_large_output_sets(dups):
    # A^12 duplicated: output sets of about dups + 10 ids inside the runs;
    # 300 copies exceed the count table's 8-bit sizes (general walk)
    inst = _instance(500 + dups, 200_011, dups)
    d = ac.ac_build(inst.patterns, sigma=4, hot_states=200)
    _say("dups", dups, "max output", d.info.max_output)
    total = _check(inst, d, {"placement": ac.AC_PLACE_HYBRID})
    _check(inst, d, {"placement": ac.AC_PLACE_HYBRID, "chains": 1})
    # a capacity that ends inside the dense runs: the canonical prefix
    _check(inst, d, {"placement": ac.AC_PLACE_HYBRID}, capacity=total // 2 + 3)


def test_hybrid_overflow_writes_nothing_past_capacity():
    torch = torch_cuda()
    inst = _instance(77, 150_001, dups=40)
    d = ac.ac_build(inst.patterns, sigma=4, hot_states=100)
    t = device_text(inst, ac.AC_TEXT_2BIT)
    want = oracle.Machine(inst.patterns, 4).scan_keys(inst.text)
    for cap in (1, len(want) // 3, len(want) - 1):
        out = torch.full((cap + 64, 2), -1, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        ac.ac_scan(d, t, len(inst.text), ac.AC_TEXT_2BIT, out, cap, cnt,
                   tune={"placement": ac.AC_PLACE_HYBRID})
        torch.cuda.synchronize()
        _say("capacity", cap, "of", len(want))
        assert int(cnt.item()) == len(want)
        assert np.array_equal(ac.match_keys(out[:cap]), want[:cap])
        assert (out[cap:] == -1).all()


@pytest.mark.parametrize("hot", [0, 50, 2000])
def test_hybrid_walk_long_patterns(hot):
    # patterns of 34-200 bases: the warm-up before each chunk spans more
    # than two 16-base text words, the walk's other warm-up path; chunks of
    # 64 are shorter than the longest pattern
    rng = W.rng_for(900 + hot)
    n = 120_007
    text = rng.integers(0, 4, size=n, dtype=np.uint8)
    for start in range(100, n - 300, 9000):
        text[start:start + int(rng.integers(40, 260))] = 0
    pats = W._cut(rng, text, rng.integers(34, 201, size=120))
    pats += [np.zeros(k, np.uint8) for k in (34, 40, 64, 100, 200)]
    pats += [rng.integers(0, 4, size=int(L), dtype=np.uint8) for L in rng.integers(34, 80, size=60)]
    pats += W._cut(rng, text, rng.integers(6, 12, size=40))      # short ones too
    inst = W.Instance(text, W.PatternSet.from_list(pats), 4, W.DNA, "long")
    d = ac.ac_build(inst.patterns, sigma=4, hot_states=hot)
    assert d.info.max_len >= 34
    for chains in (1, 2, 4):
        for chunk in (64, 256):
            tune = {"placement": ac.AC_PLACE_HYBRID, "chains": chains, "chunk": chunk}
            _say("long patterns, hot rows", hot, "tune", tune)
            _check(inst, d, tune)
