"""The built library loads and exports every function include/lqcd.h declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqcd.h")
LIB = os.path.join(ROOT, "paper_1903_06986_amd", "liblqcd.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:lqcd_status|void|const char\s*\*)\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_six_calls():
    names = declared_functions()
    for n in ("wilson_apply", "gmresdr_solve", "deflate_project", "pert_subtract",
              "poly_subtract", "loop_estimate"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblqcd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblqcd.so not built")
def test_invalid_arguments_are_reported_without_a_gpu_call():
    from paper_1903_06986_amd import lqcd
    L = lqcd.lib()
    out = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(4, 4, 3, 4)
    code = L.lqcd_create(dims, None, 0.1, None, ctypes.byref(out))
    assert code == 1 and out.value is None
    dims = (ctypes.c_int * 4)(4, 4, 3, 4)
    code = L.lqcd_create(dims, ctypes.c_void_p(1), 0.1, None, ctypes.byref(out))
    assert code == 1
    assert b"even" in L.lqcd_last_error()


def test_binding_rejects_fields_of_the_wrong_type_or_size():
    """The binding checks every field's dtype and element count before a
    pointer reaches the library (a mismatch would let kernels run past the
    allocation); host tensors are rejected as well."""
    import torch
    from paper_1903_06986_amd.lqcd import _field
    with pytest.raises(ValueError, match="dtype"):
        _field(torch.zeros(2 * 12 * 16, dtype=torch.complex64), 2, 12 * 16, "eta")
    with pytest.raises(ValueError, match="elements"):
        _field(torch.zeros(12 * 16, dtype=torch.complex128), 2, 12 * 16, "eta")
    with pytest.raises(ValueError, match="GPU"):
        _field(torch.zeros(2 * 12 * 16, dtype=torch.complex128), 2, 12 * 16, "eta")
    with pytest.raises(TypeError):
        _field([0.0], 1, 1, "eta")
