"""Build the HIP library libac.so for gfx950, in-tree.

    python -m paper_1403_7294_amd.build        (or build() from Python)

Host sources are compiled by g++, the HIP source by hipcc for gfx950 only,
and everything is linked into paper_1403_7294_amd/libac.so.  The roofline
microbenchmarks (csrc/microbench.hip) become libac_microbench.so, which only
the benchmark loads.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libac.so")
MB_LIB = os.path.join(HERE, "libac_microbench.so")  # roofline denominators (bench only)
OBJ = os.path.join(HERE, "_build")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

HOST_SOURCES = ["automaton.cpp", "api.cpp", "serve.cpp"]
HIP_SOURCES = ["scan.hip", "sort.hip"]
MB_SOURCES = ["microbench.hip"]
DEPS = ["internal.h", "batch.inc", "device_common.h"]

# packed fp32 instructions are disabled on every HIP compile (they are never
# needed here and are kept out of the code objects on purpose)
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
             "-munsafe-fp-atomics"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-I", INCLUDE,
              "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose: bool = False, extra_hip_flags=()) -> str:
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        _run(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in HIP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        out = _run([HIPCC] + HIP_FLAGS + list(extra_hip_flags) +
                   ["-c", os.path.join(CSRC, src), "-o", o])
        if verbose and out.strip():
            print(out)
        objs.append(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    mb_objs = []
    for src in MB_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        _run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o])
        mb_objs.append(o)
    tmp = MB_LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + mb_objs)
    os.replace(tmp, MB_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
