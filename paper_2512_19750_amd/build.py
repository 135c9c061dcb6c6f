"""Build libgace.so (the probe library) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgace.so")
SOURCES = ["csrc/kernels.hip", "csrc/compile.cpp", "csrc/runtime.cpp", "csrc/server.cpp", "csrc/gate.cpp", "csrc/hostpath.cpp", "csrc/estimate.cpp", "csrc/zonemap.cpp",
           "csrc/noalloc.hip"]
HIPCC = "/opt/rocm/bin/hipcc"
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17", "-Wall",
         # packed fp32 instructions stay disabled in all device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-lpthread"]


def source_hash() -> str:
    """Hash of every library source: names the kernels a tuned schedule was measured on."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(os.path.join(HERE, "csrc"))):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, '-DGACE_SOURCE_HASH="%s"' % source_hash(), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
