"""Build the gfx950 shared library libqhp.so in this package directory.

    python -m paper_2312_06367_amd.build        (or build() from Python)
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libqhp.so")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep packed FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware FP64 atomic add on device (coarse-grained) memory
    "-munsafe-fp-atomics",
    "-Wno-unused-command-line-argument",
]


def sources():
    csrc = os.path.join(HERE, "csrc")
    return sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.cpp")))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + sources() + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    # every symbol of the library's own namespace must be defined inside it: a
    # kernel template whose host pass is dropped links but cannot be loaded
    und = subprocess.run(["nm", "-D", "--undefined-only", tmp], check=True, capture_output=True, text=True).stdout
    missing = [ln.split()[-1] for ln in und.splitlines() if "_ZN3qhp" in ln]
    if missing:
        os.remove(tmp)
        raise RuntimeError("libqhp.so leaves %d symbols of namespace qhp undefined, e.g. %s" % (len(missing), missing[0]))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
