"""The pins are strong enough: plausible mistakes planted in a copy of the
oracle's source (compiled on the CPU, never used elsewhere) each make at least
one pin fail."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W
from conftest import ROOT

SRC = os.path.join(ROOT, "oracle", "ac_oracle.c")
NAIVE = os.path.join(ROOT, "oracle", "naive.c")

MUTANTS = {
    # out(s) keeps only the keywords ending at s (drops out(f(s)))
    "no_output_inheritance": ("if (inh->len == 0) continue;", "continue;"),
    # failure search restarts at the root instead of following f(r)
    "failure_from_root": ("int32_t t = m->fail[r];", "int32_t t = 0;"),
    # off-by-one end position
    "end_plus_one": ("end[total] = (uint32_t)e;", "end[total] = (uint32_t)(e + 1);"),
    # failure link of a child set to its parent's failure state
    "fail_to_parent_fail": ("m->fail[s] = m->go[(size_t)t * sigma + a];",
                            "m->fail[s] = t;"),
    # output merge takes inherited ids first (breaks the (end, id) order)
    "merge_order": ("own->ids[x] < inh->ids[y]", "own->ids[x] > inh->ids[y]"),
}


def _build_mutant(tmp_path, name):
    before, after = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(before) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(before, after))
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-o", str(so), str(path), NAIVE],
                   check=True)
    return oracle._open(str(so))


def _pins_pass(lib):
    """A fast subset of the pins; returns False as soon as one fails."""
    saved = oracle._lib
    oracle._lib = lib
    try:
        # worked example: HIS, HERS, SHE over SHERS
        alpha = "EHIRS"
        pats = [[alpha.index(c) for c in p] for p in ("HIS", "HERS", "SHE")]
        m = oracle.Machine(pats, 5)
        t = np.array([alpha.index(c) for c in "SHERS"], dtype=np.uint8)
        if m.trace(t) != [("g", 7), ("g", 8), ("g", 9), ("f", 4), ("g", 5), ("g", 6)]:
            return False
        pid, end = m.scan(t)
        if list(zip(pid.tolist(), end.tolist())) != [(2, 2), (1, 4)]:
            return False
        # brute force on tiny inputs
        for seed in range(300):
            inst = W.tiny(seed, 3)
            got = oracle.Machine(inst.patterns, 3).scan(inst.text)
            want = oracle.naive_scan(inst.text, inst.patterns)
            if not (np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])):
                return False
        return True
    except Exception:
        return False
    finally:
        oracle._lib = saved


def test_unmutated_copy_passes(tmp_path):
    so = tmp_path / "libsame.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-o", str(so), SRC, NAIVE],
                   check=True)
    assert _pins_pass(oracle._open(str(so)))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_build_mutant(tmp_path, name))
