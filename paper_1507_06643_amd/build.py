"""Build libdpde.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "api.hip")
LIB = os.path.join(HERE, "libdpde.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # expression-level contraction only: the same source expression gives the
    # same instructions in both SER sweeps
    "-ffp-contract=on",
    # keep hipcc from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def _generic_hip_soname(path: str) -> None:
    """Record the HIP runtime dependency under its generic name.

    hipcc links against /opt/rocm/lib/libamdhip64.so, whose SONAME carries
    the major version (libamdhip64.so.7).  A process that already holds a HIP
    runtime loaded under the generic name libamdhip64.so (PyTorch ships its
    own copy) would then map a second, independent runtime: separate device
    state and stream handles that are not valid across the two.  Rewriting
    the NEEDED string (same length, NUL padded) makes the loader reuse the
    runtime already present; a process without one resolves the generic name
    through the run path to /opt/rocm/lib.
    """
    data = bytearray(open(path, "rb").read())
    old, new = b"libamdhip64.so.7\x00", b"libamdhip64.so\x00\x00\x00"
    count = data.count(old)
    if count != 1:
        raise RuntimeError(f"expected one {old!r} in {path}, found {count}")
    i = data.index(old)
    data[i:i + len(old)] = new
    open(path, "wb").write(bytes(data))


def build(verbose: bool = False) -> str:
    cmd = [HIPCC] + FLAGS + ["-Wl,-rpath,/opt/rocm/lib", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    _generic_hip_soname(LIB + ".tmp")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
