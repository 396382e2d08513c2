"""Build liblrq.so (HIP kernels + C ABI + host SA builder) for gfx950, in-tree.

    python -m paper_1501_06663_amd.build

The library is written next to this file.  Both sources are compiled by hipcc
with packed FP32 instructions disabled (the kernels are integer code; the flag
keeps the compiler from pairing any float arithmetic).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblrq.so")
SOURCES = [os.path.join(HERE, "csrc", "lrq_device.hip"), os.path.join(HERE, "csrc", "lrq_host.cpp")]
PROBE_LIB = os.path.join(HERE, "libprobe.so")
PROBE_SOURCES = [os.path.join(HERE, "csrc", "probe.hip")]
ARCH = os.environ.get("LRQ_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(lib: str, sources, verbose: bool) -> str:
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-fopenmp", "-Wall", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
           "-o", tmp] + list(sources)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """liblrq.so (the query path) and libprobe.so (bench microbenchmarks)."""
    _compile(PROBE_LIB, PROBE_SOURCES, verbose)
    return _compile(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
