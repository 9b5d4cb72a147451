"""CPU checks of the C ABI: the library builds for gfx950, loads, and exports
every function include/hom.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hom.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(hom_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_and_binding_agree():
    from paper_1311_0089_amd import EXPORTED_SYMBOLS
    assert sorted(EXPORTED_SYMBOLS) == declared_functions()


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_1311_0089_amd", "libhom.so")
    if not os.path.exists(path):
        pytest.skip("libhom.so not built")
    L = ctypes.CDLL(path)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings_and_defaults():
    path = os.path.join(ROOT, "paper_1311_0089_amd", "libhom.so")
    if not os.path.exists(path):
        pytest.skip("libhom.so not built")
    from paper_1311_0089_amd import hom
    L = hom.lib()
    assert L.hom_status_str(0) == b"ok"
    assert L.hom_status_str(-4) == b"not converged"
    o = hom.Options()
    assert L.hom_options_default(ctypes.byref(o)) == 0
    assert o.scheme == 0 and o.prec == 0 and o.Y[0] == 0.5 and o.max_iter > 0
    assert L.hom_options_default(None) == -1


def test_invalid_arguments_rejected_before_device_use():
    """Argument checks run on the host before any HIP call."""
    path = os.path.join(ROOT, "paper_1311_0089_amd", "libhom.so")
    if not os.path.exists(path):
        pytest.skip("libhom.so not built")
    from paper_1311_0089_amd import hom
    L = hom.lib()
    out = ctypes.c_void_p()
    A = (ctypes.c_double * 16)(*([1.0] * 16))
    for d, N in [(2, (4, 5, 1)), (0, (5, 5, 1)), (4, (5, 5, 5)), (2, (5, 0, 1))]:
        Nc = (ctypes.c_int32 * 3)(*N)
        assert L.hom_create_cell(d, Nc, 0, A, 0, None, ctypes.byref(out)) == -1
    Nc = (ctypes.c_int32 * 3)(3, 3, 1)
    assert L.hom_create_cell(2, Nc, 7, A, 0, None, ctypes.byref(out)) == -1
    assert L.hom_solve(None, 1, None, 1e-6, None, None, None, None, None) == -1
