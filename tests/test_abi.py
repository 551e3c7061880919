"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/stkfmm.h, and answers the pure host queries."""
import ctypes
import os
import re

import pytest

import paper_2010_15155_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "stkfmm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stkfmm_[a-z_]+)\s*\(", text)))


def test_header_lists_binding_symbols():
    assert header_functions() == sorted(pkg.SYMBOLS)


def test_library_exports_every_symbol():
    L = pkg.lib()
    for name in header_functions():
        assert hasattr(L, name), name


@pytest.mark.parametrize("kernel,dims", [("LapPGrad", (1, 3, 4)), ("Stokeslet", (3, 0, 3)),
                                         ("RPY", (4, 0, 6)), ("PVel", (4, 9, 4)),
                                         ("Traction", (4, 9, 9)), ("StokesRegVel", (4, 0, 3)),
                                         ("StokesRegVelOmega", (7, 0, 6)), ("LapPGradGrad", (1, 3, 10)),
                                         ("PVelGrad", (4, 9, 16)), ("PVelLaplacian", (4, 9, 7)),
                                         ("LapQPGradGrad", (9, 0, 10))])
def test_kernel_dims(kernel, dims):
    # widths of the appendix table of supported kernels
    assert pkg.kernel_dims(kernel) == dims


def test_kernel_dims_rejects_bad_input():
    L = pkg.lib()
    a = ctypes.c_int()
    assert L.stkfmm_kernel_dims(99, ctypes.byref(a), ctypes.byref(a), ctypes.byref(a)) == 1
    assert L.stkfmm_kernel_dims(1, None, ctypes.byref(a), ctypes.byref(a)) == 1


def test_null_context_is_rejected():
    L = pkg.lib()
    assert L.stkfmm_run(None, None, None, None, None) == 1
    assert L.stkfmm_direct_noalloc(None, 1, 0, None, None, 0, None, None, 0, None, None, None) == 1
    assert L.stkfmm_set_option(None, b"precision", b"fp32") == 1
    assert L.stkfmm_last_error(None) == b"null context"
    L.stkfmm_destroy(None)
