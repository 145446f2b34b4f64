"""Build libqvts.so, the gfx950 HIP library behind the C ABI in include/qvts.h.

Run as ``python -m paper_1810_00204_amd.build``; ``__graft_entry__.build()``
calls :func:`build`.  The library is written next to this file, in-tree.
"""
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libqvts.so")
ARCH = os.environ.get("QVTS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# roctx ranges for rocprofv3's marker trace (QVTS_ROCTX=1)
LIBS = ["-lrocprofiler-sdk-roctx"]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def source_hash() -> str:
    """Hash of every file under csrc/ (kernels, headers): measurements taken
    on one build are tagged with it."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-o", tmp] + sources() + LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
