"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/blockoa.h declares, and rejects bad arguments before
launching anything."""
import ctypes
import os
import re

import pytest

from paper_2510_23221_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names.update(re.findall(r"\b(bko_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("bko_assemble_heat_operator", "bko_block_krylov_solve", "bko_combine", "bko_apply_operator"):
        assert must in names
    assert set(capi.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    lib = capi.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert capi.version().startswith("blockoa")


def test_operator_bytes_and_validation():
    lib = capi.load_library()
    out = ctypes.c_size_t()
    assert lib.bko_operator_bytes(128, 128, 8, ctypes.byref(out)) == capi.OK
    n = 128 * 128 * 8
    assert out.value >= n * (4 * 8 + 4 * 4)
    assert lib.bko_operator_bytes(0, 4, 4, ctypes.byref(out)) == capi.EINVAL
    assert b"must be positive" in lib.bko_last_error()


def test_assemble_rejects_before_launch():
    lib = capi.load_library()
    h = ctypes.c_void_p()
    bc = (ctypes.c_int * 6)(*[capi.BC_ADIABATIC] * 6)
    hh = (ctypes.c_double * 6)(*[0.0] * 6)
    fake = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    st = lib.bko_assemble_heat_operator(4, 4, 4, 1.0, 1.0, 1.0, fake, bc, hh, fake, 1 << 20, None, ctypes.byref(h))
    assert st == capi.EINVAL and b"adiabatic" in lib.bko_last_error()
    bc2 = (ctypes.c_int * 6)(*[capi.BC_ROBIN] * 6)
    st = lib.bko_assemble_heat_operator(4, 4, 4, 1.0, 1.0, 1.0, fake, bc2, hh, fake, 1 << 20, None, ctypes.byref(h))
    assert st == capi.EINVAL and b"Robin" in lib.bko_last_error()
    bc3 = (ctypes.c_int * 6)(*[7] * 6)
    st = lib.bko_assemble_heat_operator(4, 4, 4, 1.0, 1.0, 1.0, fake, bc3, hh, fake, 1 << 20, None, ctypes.byref(h))
    assert st == capi.EINVAL
    bc4 = (ctypes.c_int * 6)(*[capi.BC_DIRICHLET0] * 6)
    st = lib.bko_assemble_heat_operator(4, 4, 4, 1.0, 1.0, 1.0, fake, bc4, hh, fake, 16, None, ctypes.byref(h))
    assert st == capi.EINVAL and b"need" in lib.bko_last_error()
    st = lib.bko_assemble_heat_operator(4, 4, 4, -1.0, 1.0, 1.0, fake, bc4, hh, fake, 1 << 20, None, ctypes.byref(h))
    assert st == capi.EINVAL


def test_combine_validation():
    lib = capi.load_library()
    fake = ctypes.c_void_p(256)
    # s beyond the supported maximum
    assert lib.bko_combine(10, 65, 3, fake, 10, 0, fake, 65, 0, fake, 10, 0, 0, None) == capi.EINVAL
    # leading dimension too small
    assert lib.bko_combine(10, 4, 3, fake, 9, 0, fake, 4, 0, fake, 10, 0, 0, None) == capi.EINVAL
    # bad dtype code
    assert lib.bko_combine(10, 4, 3, fake, 10, 9, fake, 4, 0, fake, 10, 0, 0, None) == capi.EINVAL
    # empty work is a no-op
    assert lib.bko_combine(0, 4, 3, fake, 10, 0, fake, 4, 0, fake, 10, 0, 0, None) == capi.OK


def test_solve_and_apply_reject_null_handle():
    lib = capi.load_library()
    info = capi.SolveInfo()
    fake = ctypes.c_void_p(256)
    assert lib.bko_block_krylov_solve(None, 4, fake, 10, fake, 10, None, 0, 0, 1e-8, 10, fake, 1 << 20,
                                      ctypes.byref(info), None) == capi.EINVAL
    assert lib.bko_apply_operator(None, 4, fake, 10, 0, fake, 10, 0, 0, None) == capi.EINVAL
    n = ctypes.c_size_t()
    assert lib.bko_block_krylov_workspace_bytes(None, 4, 0, ctypes.byref(n)) == capi.EINVAL
    assert lib.bko_timing_query(99, None, None) == capi.EINVAL


def test_no_cpu_fallback(monkeypatch, tmp_path):
    """The binding refuses to run without the built library."""
    monkeypatch.setattr(capi, "_lib", None)
    with pytest.raises(ImportError):
        capi.load_library(str(tmp_path / "missing.so"))


def test_copy_rejects_before_launch():
    lib = capi.load_library()
    a, b = ctypes.c_void_p(4096), ctypes.c_void_p(1 << 20)  # never dereferenced
    assert lib.bko_copy(b, a, 24, None) == capi.EINVAL  # not a multiple of 16 bytes
    assert lib.bko_copy(ctypes.c_void_p(4104), a, 32, None) == capi.EINVAL  # misaligned
    assert lib.bko_copy(ctypes.c_void_p(4096 + 16), a, 64, None) == capi.EINVAL  # overlap
    assert b"overlap" in lib.bko_last_error()
    assert lib.bko_copy(b, a, 0, None) == capi.OK  # nothing to do
