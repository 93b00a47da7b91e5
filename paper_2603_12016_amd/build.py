"""Build step for libnyx.so: hipcc for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/nyx_kernels.hip", "csrc/nyx_intensity.hip", "csrc/nyx_neighbourhood.hip", "csrc/nyx_runtime.hip"]
HEADERS = ["csrc/nyx_types.h", "csrc/nyx_device.h", "csrc/nyx_features.h", "csrc/nyx_launch.h"]
LIB = os.path.join(HERE, "libnyx.so")
MICRO_SOURCES = ["csrc/nyx_micro.hip"]
MICRO_LIB = os.path.join(HERE, "libnyx_micro.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _compile(sources, lib, verbose):
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, "-I" + os.path.join(HERE, "csrc"), "-I" + os.path.join(ROOT, "include"),
           "-o", tmp, *[os.path.join(HERE, s) for s in sources]]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Compile libnyx.so and the measurement kernels libnyx_micro.so (always recompiles)."""
    _compile(MICRO_SOURCES, MICRO_LIB, verbose)
    return _compile(SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
