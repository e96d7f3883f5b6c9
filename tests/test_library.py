"""Host-side checks of the HIP library: it loads and exports every symbol that
include/rbfgs.h declares (no compute calls; runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbfgs.h")
LIB = os.path.join(ROOT, "paper_1602_01768_amd", "librbfgs.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbfgs_[a-z_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_header():
    from paper_1602_01768_amd import rbfgs
    assert set(declared_symbols()) <= set(rbfgs.EXPORTS)
    rbfgs.load_library()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_arguments_rejected_without_gpu_work():
    """Argument validation happens before any device call."""
    from paper_1602_01768_amd import rbfgs
    lib = rbfgs.load_library()
    out = ctypes.c_void_p(123)
    p = rbfgs.rbfgs_params(n=4, q=5, seed=1, sketch=0, variant=0, precision=0, check_every=1)
    a = (ctypes.c_double * 16)()
    assert lib.rbfgs_create(ctypes.byref(p), a, 1, 4, 0, None, ctypes.byref(out)) == rbfgs.E_INVALID_ARG
    assert out.value is None
    p.q = 0
    assert lib.rbfgs_create(ctypes.byref(p), a, 1, 4, 0, None, ctypes.byref(out)) == rbfgs.E_INVALID_ARG
    p.q, p.sketch = 2, 7
    assert lib.rbfgs_create(ctypes.byref(p), a, 1, 4, 0, None, ctypes.byref(out)) == rbfgs.E_INVALID_ARG
    p.sketch = 0
    assert lib.rbfgs_create(ctypes.byref(p), a, 1, 3, 0, None, ctypes.byref(out)) == rbfgs.E_INVALID_ARG  # lda < n
    assert lib.rbfgs_create(ctypes.byref(p), None, 1, 4, 0, None, ctypes.byref(out)) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_step(None, 1) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_sketch_coord(1, 0, 5, 6, ctypes.c_void_p(16), None) == rbfgs.E_INVALID_ARG
    lib.rbfgs_destroy(None)
