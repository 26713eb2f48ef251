"""Build step of the HIP library (hipcc, gfx950).

Produces ``libmmbb.so`` next to this file from ``csrc/*.hip`` and, beside it,
``libmmbb.so.srchash``: a hash of every source file, the C header and the
compiler flags it was built from, so that a binary older than its sources
is recognised (``is_current``) and rebuilt (``ensure_built``).
"""

import hashlib
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


def hash_path():
    return lib_path() + ".srchash"


def sources_hash():
    """Hash of csrc/ (every file), include/mm.h and the compiler flags."""
    h = hashlib.sha256()
    d = os.path.join(HERE, "csrc")
    files = [os.path.join(d, f) for f in sorted(os.listdir(d))]
    files.append(os.path.join(os.path.dirname(HERE), "include", "mm.h"))
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    h.update(" ".join(FLAGS + SOURCES).encode())
    return h.hexdigest()[:16]


def is_current():
    """Whether the built library exists and was built from the present sources."""
    if not os.path.exists(lib_path()) or not os.path.exists(hash_path()):
        return False
    with open(hash_path()) as fh:
        return fh.read().strip() == sources_hash()


def ensure_built(verbose=True):
    """Rebuild the library when it is missing or older than its sources."""
    if not is_current():
        if verbose:
            print("libmmbb.so missing or built from other sources: rebuilding", flush=True)
        build(verbose=verbose)
    return lib_path()


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed with exit code %d" % res.returncode)


def build(verbose=True, jobs=None):
    """Compile every HIP source into the shared library (always rebuilds):
    one object per source, compiled in parallel, then linked."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmds.append([hipcc] + compile_flags + ["-c", "-o", obj, os.path.join(HERE, "csrc", src)])
        objs.append(obj)
    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = lib_path() + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    digest = sources_hash()
    os.replace(tmp, lib_path())
    with open(hash_path(), "w") as fh:
        fh.write(digest + "\n")
    return lib_path()


if __name__ == "__main__":
    build()
