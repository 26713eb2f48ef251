"""Build step of the HIP library (hipcc, gfx950).

Produces ``libmmbb.so`` next to this file from ``csrc/*.hip``.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["capi.hip", "demag.hip", "demag3d.hip", "tensor.hip", "local.hip", "iter.hip", "adjoint.hip"]
LIB_NAME = "libmmbb.so"

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are switched off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def lib_path():
    return os.path.join(HERE, LIB_NAME)


def build(verbose=True):
    """Compile every HIP source into the shared library (always rebuilds)."""
    hipcc = os.environ.get("HIPCC", "hipcc")
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = lib_path() + ".tmp"
    cmd = [hipcc] + FLAGS + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed with exit code %d" % res.returncode)
    os.replace(tmp, lib_path())
    return lib_path()


if __name__ == "__main__":
    build()
