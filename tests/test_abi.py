"""The C ABI library loads, exports every function include/wd.h declares, and
rejects invalid arguments before touching the device (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(\w+)\s*\([^;{]*\)\s*;", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_0911_3191_amd as wd
    return wd.lib()


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for n in ("wilson_dslash", "mdagm", "wilson_mat_pc", "bicgstab_solve", "cg_solve", "wd_gauge_create",
              "wd_spinor_encode", "wd_operator_workspace_bytes", "wd_dslash_field", "wd_dslash_field_basis",
              "wd_mat_pc_field", "wd_mdagm_field", "wd_spinor_encode_basis", "wd_spinor_decode_basis"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_validation_rejects_bad_lattices_and_arguments(lib):
    import paper_0911_3191_amd as wd
    assert wd.wd_gauge_bytes(wd.lattice((4, 4, 4, 3)), 1) == 0       # odd dim
    assert wd.wd_gauge_bytes(wd.lattice((0, 4, 4, 4)), 1) == 0       # empty
    assert wd.wd_gauge_bytes(wd.lattice((4, 4, 4, 4)), 0) == 0       # empty mask
    assert wd.wd_spinor_bytes(wd.lattice((4, 4, 4, 4)), "fp32", 0) == 0
    n64 = wd.wd_spinor_bytes(wd.lattice((4, 4, 4, 4)), "fp64", 1)
    assert n64 == 12 * 128 * 16
    assert wd.wd_spinor_bytes(wd.lattice((4, 4, 4, 4)), "i16", 2) == 2 * (3 * 128 * 16 + 128 * 4)
    # NULL gauge handle and NULL fields are refused with WD_EINVAL, no launch
    st = lib.wd_dslash_field(None, None, None, 0, 0, 0, 1, None)
    assert st == -1
    assert b"NULL" in lib.wd_last_error()
    lat = wd.lattice((4, 4, 4, 4))
    h = ctypes.c_void_p()
    st = lib.wd_gauge_create(ctypes.byref(lat), ctypes.c_void_p(256), 1, ctypes.c_void_p(512), 10,
                             None, ctypes.byref(h))
    assert st == -1 and b"too small" in lib.wd_last_error()
    # device pointers must be 256-byte aligned
    for bad_ptr in (17, 16, 128):
        st = lib.wd_gauge_create(ctypes.byref(lat), ctypes.c_void_p(bad_ptr), 1, ctypes.c_void_p(512), 1 << 30,
                                 None, ctypes.byref(h))
        assert st == -1 and b"256-byte aligned" in lib.wd_last_error()
    bad = wd.lattice((4, 4, 4, 5))
    st = lib.wd_spinor_encode(ctypes.byref(bad), 0, 1, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert st == -1 and b"even" in lib.wd_last_error()
    # an unknown spin basis is refused before any launch
    for fn in (lib.wd_spinor_encode_basis, lib.wd_spinor_decode_basis):
        st = fn(ctypes.byref(lat), 0, 1, 2, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
        assert st == -1 and b"basis" in lib.wd_last_error()
    st = lib.wd_dslash_field_basis(None, None, None, 0, 0, 0, 1, 1, None)
    assert st == -1 and b"NULL" in lib.wd_last_error()


def test_lattices_beyond_the_32_bit_descriptor_range_are_refused(lib):
    """One FP64 parity field of one RHS must stay below 4 GiB (the kernels'
    buffer descriptors carry a 32-bit size): the largest accepted Vh is
    22,369,600; 64^3 x 192 (Vh = 25,165,824) is refused, 64^3 x 160 is not."""
    import paper_0911_3191_amd as wd
    big = wd.lattice((64, 64, 64, 192))
    assert wd.wd_spinor_bytes(big, "f16", 1) == 0
    assert wd.wd_gauge_bytes(big, 1 << 3) == 0
    assert wd.wd_operator_workspace_bytes(big, "fp32", 1) == 0
    st = lib.wd_spinor_encode(ctypes.byref(big), 3, 1, ctypes.c_void_p(256), ctypes.c_void_p(256), None)
    assert st == -1 and b"too large" in lib.wd_last_error()
    ok = wd.lattice((64, 64, 64, 160))
    vh = 64 ** 3 * 160 // 2
    assert vh <= 22369600
    assert wd.wd_spinor_bytes(ok, "fp64", 1) == 12 * 16 * ((vh + 63) // 64 * 64)
    assert wd.wd_spinor_bytes(ok, "fp64", 1) < 2 ** 32
    # the boundary case: the largest stride that fits
    edge = wd.lattice((2, 2, 2, 2 * 22369600 // 8))
    assert wd.wd_spinor_bytes(edge, "fp64", 1) == 192 * 22369600
    over = wd.lattice((2, 2, 2, 2 * 22369600 // 8 + 32))
    assert wd.wd_spinor_bytes(over, "fp64", 1) == 0


def test_canonical_operators_validate_before_any_launch(lib):
    """wilson_dslash / wilson_mat_pc / mdagm on canonical FP64 spinors take a
    workspace of wd_operator_workspace_bytes: four encoded fields, each
    rounded up to 256 bytes."""
    import paper_0911_3191_amd as wd
    lat = wd.lattice((4, 4, 4, 4))
    for prec, nrhs in (("fp64", 1), ("fp32", 3), ("i16", 2), ("f16", 12)):
        n = wd.wd_spinor_bytes(lat, prec, nrhs)
        assert wd.wd_operator_workspace_bytes(lat, prec, nrhs) == 4 * ((n + 255) // 256 * 256)
    assert wd.wd_operator_workspace_bytes(lat, "fp32", 0) == 0
    st = lib.wilson_dslash(None, None, None, 0, 0, 0, 1, None, 0, None)
    assert st == -1 and b"NULL" in lib.wd_last_error()
    st = lib.mdagm(None, 0.12, None, None, 0, 1, None, 0, None)
    assert st == -1 and b"NULL" in lib.wd_last_error()
    st = lib.wilson_mat_pc(None, 0.12, None, None, 0, 0, 1, None, 0, None)
    assert st == -1 and b"NULL" in lib.wd_last_error()


@pytest.mark.parametrize("field,value,msg", [
    ("restart", 2, b"restart"), ("delta", 1.0, b"delta"), ("nrhs", 0, b"nrhs"), ("nrhs", 65, b"nrhs"),
    ("tol", 0.0, b"tol"),
    ("maxiter", 0, b"maxiter"), ("x0_given", 1, b"x0_given")])
def test_solver_parameters_are_validated_before_any_launch(lib, field, value, msg):
    import paper_0911_3191_amd as wd
    p = wd.solve_params(tol=1e-12, inner="f16", delta=0.1, nrhs=1)
    setattr(p, field, value)
    st = lib.bicgstab_solve(None, 0.12, None, None, ctypes.byref(p), None, None, 0, None)
    assert st in (wd.WD_EINVAL, wd.WD_EUNSUPPORTED)
    assert msg in lib.wd_last_error()


def test_defect_correction_needs_an_inner_tolerance(lib):
    import paper_0911_3191_amd as wd
    p = wd.solve_params(tol=1e-12, inner="fp32", delta=0.0, restart=True)
    st = lib.cg_solve(None, 0.12, None, None, ctypes.byref(p), None, None, 0, None)
    assert st == wd.WD_EINVAL and b"inner tolerance" in lib.wd_last_error()
