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


# Host-side sanitizer build (device code as in the library): every source
# and the driver of tests/host_sanitize/, host code instrumented with
# AddressSanitizer and UndefinedBehaviorSanitizer, linked into one program.
SAN_FLAGS = [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
    "-gline-tables-only",
]


def sanitize_driver_dir():
    return os.path.join(os.path.dirname(HERE), "tests", "host_sanitize")


def sanitize_exe():
    return os.path.join(sanitize_driver_dir(), "mm_sanitize")


def sanitize_hash():
    """Hash of the library sources plus the driver source and flags."""
    h = hashlib.sha256(sources_hash().encode())
    with open(os.path.join(sanitize_driver_dir(), "driver.cpp"), "rb") as fh:
        h.update(fh.read())
    h.update(" ".join(SAN_FLAGS).encode())
    return h.hexdigest()[:16]


def sanitize_is_current():
    exe = sanitize_exe()
    if not os.path.exists(exe) or not os.path.exists(exe + ".srchash"):
        return False
    with open(exe + ".srchash") as fh:
        return fh.read().strip() == sanitize_hash()


def build_sanitized(verbose=True, jobs=None):
    """Compile the library sources and the driver with host sanitizers into
    tests/host_sanitize/mm_sanitize (always rebuilds)."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "hipcc")
    objdir = os.path.join(HERE, "_build", "san")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"] + SAN_FLAGS
    inc = "-I" + os.path.join(os.path.dirname(HERE), "include")
    cmds, objs = [], []
    srcs = [os.path.join(HERE, "csrc", f) for f in SOURCES]
    srcs.append(os.path.join(sanitize_driver_dir(), "driver.cpp"))
    for src in srcs:
        obj = os.path.join(objdir, os.path.splitext(os.path.basename(src))[0] + ".o")
        cmds.append([hipcc] + compile_flags + [inc, "-c", "-o", obj, src])
        objs.append(obj)
    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    exe = sanitize_exe()
    _run([hipcc, "--offload-arch=gfx950"] + SAN_FLAGS + ["-o", exe + ".tmp"] + objs, verbose)
    digest = sanitize_hash()
    os.replace(exe + ".tmp", exe)
    with open(exe + ".srchash", "w") as fh:
        fh.write(digest + "\n")
    return exe


if __name__ == "__main__":
    build()
