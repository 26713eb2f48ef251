"""Host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/host_sanitize/driver.cpp calls every entry
point of include/mm.h (three grid kinds, both precisions, checkpoints,
batched, grouped and per-sample sweeps, derivatives, profiling, error paths)
in a program whose host code is instrumented (built by
__graft_entry__.build()).  It must exit 0 with no sanitizer report."""

import os
import subprocess

import pytest

from paper_1405_2728_amd import _build

pytestmark = pytest.mark.gpu


def test_host_code_is_clean_under_sanitizers():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    exe = _build.sanitize_exe()
    if not os.path.exists(exe):
        pytest.skip("sanitizer driver not built (__graft_entry__.build() builds it)")
    assert _build.sanitize_is_current(), "sanitizer driver older than its sources: rebuild"
    env = dict(os.environ)
    # leaks of the HIP runtime's own allocations are not the library's; the
    # runtime library may be loaded before the sanitizer's
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    res = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    out = res.stdout + res.stderr
    print(out[-4000:])
    assert "address sanitizer: on" in out
    assert "runtime error" not in out
    assert "AddressSanitizer" not in out
    assert res.returncode == 0
    assert "host sanitizer driver: 0 failure(s)" in out
