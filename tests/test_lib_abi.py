"""The C-ABI library loads and exports every symbol of include/mm.h; host
logic that needs no GPU (argument validation, support predicate, strings)."""

import ctypes as C
import os
import re

import pytest

from paper_1405_2728_amd import _build, _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    _build.ensure_built()
    return _lib.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mm_set_geometry", "mm_set_material", "mm_set_field", "mm_heff",
                     "mm_energy", "mm_minimize_step", "mm_minimize_to_tol",
                     "mm_hysteresis_sweep"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_support_predicate(lib):
    assert lib.mm_supported(0, 400, 200, 4) == 1       # SP1-like film
    assert lib.mm_supported(1, 400, 200, 4) == 1
    assert lib.mm_supported(0, 32, 16, 1) == 1
    assert lib.mm_supported(0, 256, 128, 2) == 1
    assert lib.mm_supported(0, 1, 1, 1) == 1
    assert lib.mm_supported(0, 0, 5, 1) == 0
    assert lib.mm_supported(0, 10, 10, 0) == 0
    # more than 4 layers: full 3-D path, y and z padded to 64..512
    assert lib.mm_supported(0, 128, 128, 128) == 1
    assert lib.mm_supported(1, 128, 128, 128) == 1
    assert lib.mm_supported(0, 1, 1, 5) == 1
    # longest x rows: 3 Px/2 complex values of a row must fit one block
    for prec in (0, 1):
        assert lib.mm_supported(prec, 2048, 3, 1) == 1     # Px 4096
        assert lib.mm_supported(prec, 2049, 3, 1) == 0     # Px 8192
        assert lib.mm_supported(prec, 2048, 8, 8) == 1     # 3-D path, same x passes
        assert lib.mm_supported(prec, 2049, 8, 8) == 0
    assert lib.mm_supported(0, 300, 256, 256) == 1
    assert lib.mm_supported(0, 8, 257, 8) == 0
    assert lib.mm_supported(0, 8, 8, 257) == 0
    assert lib.mm_supported(2, 8, 8, 8) == 0


def test_status_strings(lib):
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        assert lib.mm_strerror(code)
    assert lib.mm_kernel_name(0) == b"xf"
    assert lib.mm_kernel_name(99) is None
    names = []
    k = 0
    while lib.mm_kernel_name(k) is not None:
        names.append(lib.mm_kernel_name(k).decode())
        k += 1
    assert names == ["xf", "yz_thin", "xil", "update", "y3_fwd", "z3", "y3_inv", "finish",
                     "reference"]


def test_argument_validation_without_gpu(lib):
    h = C.c_void_p()
    assert lib.mm_create(None, 0, 1, None) == -1
    assert lib.mm_create(C.byref(h), 7, 1, None) == -1
    assert lib.mm_create(C.byref(h), 0, 0, None) == -1
    assert lib.mm_create(C.byref(h), 0, 2, None) == 0
    try:
        assert lib.mm_set_geometry(h, 0, 0, 4, 1, 1e-9, 1e-9, 1e-9) == -1
        assert lib.mm_set_geometry(h, 5, 4, 4, 1, 1e-9, 1e-9, 1e-9) == -1
        assert lib.mm_set_geometry(h, 0, 4, 4, 1, -1e-9, 1e-9, 1e-9) == -1
        assert b"cell sizes" in lib.mm_last_error(h)
        # calls before a geometry exists are out of order
        H = (C.c_double * 3)(0.0, 0.0, 0.0)
        assert lib.mm_set_field(h, 1, H) == -5
        assert lib.mm_set_material(h, 0, 8e5, 1e-11, 0.0, None, None) == -5
        assert lib.mm_set_option(h, b"poll_every", 0.0) == -1
        assert lib.mm_set_option(h, b"no_such_key", 1.0) == -1
        assert lib.mm_set_option(h, b"poll_every", 8.0) == 0
        assert lib.mm_set_option(h, b"tau0", -1.0) == -1
        assert lib.mm_set_option(h, b"demag_path", 3.0) == -1
        assert lib.mm_set_option(h, b"demag_path", 2.0) == 0
        assert lib.mm_set_option(h, b"demag_path", 0.0) == 0
        assert lib.mm_set_option(h, b"refine", 0.0) == 0
        assert lib.mm_set_option(h, b"refine", 1.0) == 0
        assert lib.mm_set_option(h, b"autotune", 1.0) == 0
        assert lib.mm_set_option(h, b"mixed_radix", 0.0) == 0
        assert lib.mm_set_option(h, b"mixed_radix", 1.0) == 0
        assert lib.mm_set_option(h, b"concurrent_groups", 0.0) == 0
        assert lib.mm_set_option(h, b"concurrent_groups", 1.0) == 0
        assert lib.mm_set_option(h, b"persistent", 0.0) == 0
        assert lib.mm_set_option(h, b"persistent", 1.0) == 0
        assert lib.mm_set_option(h, b"fused_finish", 0.0) == 0
        assert lib.mm_set_option(h, b"fused_finish", 1.0) == 0
        assert lib.mm_set_option(h, b"fin_spin", -1.0) == -1
        assert lib.mm_set_option(h, b"fin_spin", 2.5) == -1
        assert lib.mm_set_option(h, b"fin_spin", 0.0) == 0
        assert lib.mm_set_option(h, b"fin_spin", 4194304.0) == 0
        assert lib.mm_set_option(h, b"batch_rebuild", 1.0) == -1
        assert lib.mm_set_option(h, b"batch_rebuild", 0.0) == 0
        assert lib.mm_set_option(h, b"batch_rebuild", 0.75) == 0
        assert lib.mm_set_option(h, b"yz_variant", 2.0) == -1
        assert lib.mm_set_option(h, b"yz_variant", 1.0) == 0
        assert lib.mm_set_option(h, b"yz_variant", -1.0) == 0
        assert lib.mm_set_option(h, b"bb_switch", -0.5) == -1
        assert lib.mm_set_option(h, b"bb_switch", float("inf")) == -1
        assert lib.mm_set_option(h, b"bb_switch", 0.5) == 0
        assert lib.mm_set_option(h, b"bb_switch", 0.0) == 0
        assert lib.mm_set_option(h, b"line_search", 2.0) == -1
        assert lib.mm_set_option(h, b"line_search", 1.0) == 0
        assert lib.mm_set_option(h, b"line_search", 0.0) == 0
        assert lib.mm_set_option(h, b"ls_eta", 1.5) == -1
        assert lib.mm_set_option(h, b"ls_eta", 0.85) == 0
        assert lib.mm_set_option(h, b"ls_rho", 0.0) == -1
        assert lib.mm_set_option(h, b"ls_rho", 1e-4) == 0
        assert lib.mm_set_option(h, b"ls_sigma", 1.0) == -1
        assert lib.mm_set_option(h, b"ls_sigma", 0.5) == 0
        assert lib.mm_set_option(h, b"ls_max", 2.5) == -1
        assert lib.mm_set_option(h, b"ls_max", 30.0) == 0
        assert lib.mm_set_option(h, b"rows_per_block", -1.0) == -1
        assert lib.mm_set_option(h, b"rows_per_block", 2.5) == -1
        assert lib.mm_set_option(h, b"rows_per_block", 3.0) == 0
        assert lib.mm_set_option(h, b"rows_per_block", 0.0) == 0
        r = C.c_int()
        assert lib.mm_rows_per_block(h, 0, C.byref(r)) == -5
        assert lib.mm_yz_variant(h, 0, C.byref(r)) == -5
    finally:
        lib.mm_destroy(h)
    lib.mm_destroy(None)
