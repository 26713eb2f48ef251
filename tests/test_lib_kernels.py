"""Register and scratch use of the built library's kernels (no GPU needed).

The gfx950 code objects embedded in libmmbb.so carry, per kernel, the
number of VGPRs spilled to scratch memory and the fixed private-segment
(scratch) size.  A spill does not show in the register count, yet it cost
the single-precision yz pass 14% of its time and 6.9 MB of extra traffic
per launch on the 400 x 200 x 4 film.  This test keeps every kernel of the
default paths (fused x passes, wave yz pass and its persistent batched
form, 3-D y/z passes, finishes) free of VGPR spills and of any scratch use
(also non-spill scratch: a one-element array of the 64-point transforms
once stayed in scratch memory across a wave barrier), and checks the
benchmarked film and cube instances by name.
"""

import os
import re
import shutil
import struct
import subprocess

import pytest

from paper_1405_2728_amd import _build

LLVM_BIN = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"

DEFAULT_PATH = ("k_xf_w<", "k_xil_w<", "k_yz_wave<", "k_yz_wave_p<", "k_x_wp<", "k_y3_fwd<",
                "k_y3_inv<", "k_z3<", "k_w3_p<", "k_finish")

BENCHMARKED = (
    # film 400 x 200 x 4: 448-point x and y transforms, 4 layers
    "k_xf_w<double, 7, true>", "k_xil_w<double, 7>", "k_yz_wave<double, 7, 4, 3, false>",
    "k_xf_w<float, 7, true>", "k_xil_w<float, 7>", "k_yz_wave<float, 7, 4, 6, true>",
    # cube 128^3: 128-point x transforms, 256-point y and z transforms
    "k_xf_w<double, 2, false>", "k_xil_w<double, 2>", "k_y3_fwd<double, 4, false>",
    "k_z3<double, 4, false>", "k_y3_inv<double, 4, false>",
)


def _tool(name):
    path = os.path.join(LLVM_BIN, name)
    return path if os.path.exists(path) else shutil.which(name)


def _code_objects(lib_bytes):
    """gfx950 code objects of every clang offload bundle in the library."""
    out = []
    pos = lib_bytes.find(MAGIC)
    while pos != -1:
        n = struct.unpack_from("<Q", lib_bytes, pos + 24)[0]
        off = pos + 32
        for _ in range(n):
            o, size, idlen = struct.unpack_from("<QQQ", lib_bytes, off)
            tid = lib_bytes[off + 24:off + 24 + idlen].decode()
            off += 24 + idlen
            if "gfx950" in tid:
                out.append(lib_bytes[pos + o:pos + o + size])
        pos = lib_bytes.find(MAGIC, pos + 1)
    return out


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    readelf, cxxfilt = _tool("llvm-readelf"), _tool("llvm-cxxfilt") or _tool("c++filt")
    if not readelf or not cxxfilt:
        pytest.skip("llvm-readelf / c++filt not available")
    _build.ensure_built()
    with open(_build.lib_path(), "rb") as fh:
        cos = _code_objects(fh.read())
    assert cos, "no gfx950 code object in the library"
    d = tmp_path_factory.mktemp("co")
    rec = {}
    for i, co in enumerate(cos):
        p = d / ("k%d.co" % i)
        p.write_bytes(co)
        notes = subprocess.run([readelf, "--notes", str(p)], capture_output=True, text=True,
                               check=True).stdout
        cur = None
        for line in notes.splitlines():
            m = re.match(r"\s+\.name:\s+(\S+)", line)
            if m:
                cur = m.group(1)
                rec.setdefault(cur, {})
                continue
            m = re.match(r"\s+\.(vgpr_spill_count|private_segment_fixed_size):\s+(\d+)", line)
            if m and cur is not None:
                rec[cur][m.group(1)] = int(m.group(2))
    names = sorted(rec)
    dem = subprocess.run([cxxfilt], input="\n".join(names), capture_output=True, text=True,
                         check=True).stdout.splitlines()
    out = {}
    for mangled, readable in zip(names, dem):
        key = readable.split("(")[0].replace("void ", "").replace("mmk::", "").strip()
        out[key] = rec[mangled]
    return out


def test_default_path_kernels_use_no_scratch(kernels):
    hot = {k: v for k, v in kernels.items() if k.startswith(DEFAULT_PATH)}
    assert len(hot) > 50
    spilled = {k: v["vgpr_spill_count"] for k, v in hot.items() if v.get("vgpr_spill_count", 0)}
    assert not spilled, spilled
    scratch = {k: v["private_segment_fixed_size"] for k, v in hot.items()
               if v.get("private_segment_fixed_size", 0)}
    assert not scratch, scratch


def test_benchmarked_instances_use_no_scratch(kernels):
    for name in BENCHMARKED:
        assert name in kernels, name
        rec = kernels[name]
        assert rec.get("vgpr_spill_count", 0) == 0, (name, rec)
        assert rec.get("private_segment_fixed_size", 0) == 0, (name, rec)
