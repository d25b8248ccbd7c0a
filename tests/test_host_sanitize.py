"""The host half of the library (stage 1 of section III.A and the C-ABI
entry points that need no GPU) built with AddressSanitizer,
UndefinedBehaviorSanitizer and leak checking, with stand-ins for the GPU
half, and driven by tests/sanitize/host_driver.cpp:

* the tiny corpus (alphabets of 2-4 symbols, nested and duplicated
  patterns) plus shrunk DNA and protein workloads: the exported tables walked
  with the chunk/overlap rule equal the oracle for several chunk sizes,
  serial and threaded builds, and the partitioned build;
* every argument error returns its status code;
* AC_TEST_FAIL_ALLOC=<n> fails the n-th checked allocation: every n gives
  AC_E_NOMEM or AC_OK, never a crash or a leak, until no check is left.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import workloads as W
from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1403_7294_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("no host compiler")
    d = tmp_path_factory.mktemp("san")
    objs = []
    for src in ("ac_oracle.c", "naive.c"):
        o = str(d / (src + ".o"))
        subprocess.run(["gcc", "-std=c99"] + SAN + ["-c", os.path.join(ROOT, "oracle", src),
                                                    "-o", o], check=True)
        objs.append(o)
    srcs = [os.path.join(CSRC, "automaton.cpp"), os.path.join(CSRC, "api.cpp"),
            os.path.join(ROOT, "tests", "sanitize", "device_stubs.cpp"),
            os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")]
    exe = str(d / "host_driver")
    subprocess.run(["g++", "-std=c++17", "-pthread"] + SAN +
                   ["-I", os.path.join(ROOT, "include")] + srcs + objs + ["-o", exe],
                   check=True)
    return exe


def _run(exe, *args, env=None):
    e = dict(os.environ)
    e.pop("AC_TEST_FAIL_ALLOC", None)
    e["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=23"
    e["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    e.update(env or {})
    return subprocess.run([exe] + list(args), stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                          text=True, env=e, timeout=600)


def _write_corpus(path, insts):
    with open(path, "wb") as f:
        f.write(struct.pack("<I", len(insts)))
        for inst in insts:
            t = np.ascontiguousarray(inst.text, dtype=np.uint8)
            f.write(struct.pack("<II", inst.sigma, len(t)))
            f.write(t.tobytes())
            off = np.ascontiguousarray(inst.patterns.offsets, dtype=np.uint64)
            f.write(struct.pack("<I", len(off) - 1))
            f.write(off.tobytes())
            f.write(np.ascontiguousarray(inst.patterns.symbols[:int(off[-1])],
                                         dtype=np.uint8).tobytes())


def test_corpus_under_sanitizers(driver, tmp_path):
    insts = [W.tiny(seed, sigma) for sigma in (2, 3, 4) for seed in range(120)]
    insts += [W.dna_small(scale=1 / 64), W.protein(scale=1 / 4096),
              W.dna_dense(scale=1 / 4096)]        # 10,000 patterns: the threaded build
    path = str(tmp_path / "corpus.bin")
    _write_corpus(path, insts)
    r = _run(driver, "corpus", path)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.startswith(f"ok {len(insts)} instances")


def test_argument_errors_under_sanitizers(driver):
    r = _run(driver, "errors")
    assert r.returncode == 0, r.stderr[-3000:] + r.stdout


def test_allocation_failures_release_everything(driver):
    r = _run(driver, "alloc")
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.split() == ["0", "0"]
    failed = 0
    for n in range(1, 64):
        r = _run(driver, "alloc", env={"AC_TEST_FAIL_ALLOC": str(n)})
        assert r.returncode == 0, (n, r.stderr[-3000:])       # no crash, no leak
        a, b = (int(x) for x in r.stdout.split())
        assert a in (0, -5) and b in (0, -5), (n, a, b)
        failed += (a == -5) + (b == -5)
        if a == 0 and b == 0:
            break
    else:
        pytest.fail("allocation checks never ran out")
    assert failed >= 6          # the build's and the partitioned build's checks were all hit
