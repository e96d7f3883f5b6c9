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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_sketch_and_variant_combinations_validated_on_host():
    """Partition sampling needs fixed RBFGS or AdaRBFGS and q | n; importance sampling needs
    Kaczmarz and q | n; Newton-Schulz and MR run in FP64 only; unknown kinds are rejected.
    All of it is decided before any device call."""
    from paper_1602_01768_amd import rbfgs
    lib = rbfgs.load_library()
    a = (ctypes.c_double * 64)()
    out = ctypes.c_void_p()

    def create(sketch, variant, precision=0, n=8, q=4):
        p = rbfgs.rbfgs_params(n=n, q=q, seed=1, sketch=sketch, variant=variant, precision=precision, check_every=1)
        return lib.rbfgs_create(ctypes.byref(p), a, 1, n, 0, None, ctypes.byref(out))

    S, V = rbfgs.SKETCH, rbfgs.VARIANT
    for variant in ("psb", "aip", "kaczmarz", "newton_schulz", "mr"):
        assert create(S["partition"], V[variant]) == rbfgs.E_INVALID_ARG, variant
    for variant in ("fixed", "adaptive", "psb", "aip", "newton_schulz", "mr"):
        assert create(S["importance"], V[variant]) == rbfgs.E_INVALID_ARG, variant
    assert create(S["partition"], V["fixed"], q=3) == rbfgs.E_INVALID_ARG      # 3 does not divide 8
    assert create(S["importance"], V["kaczmarz"], q=3) == rbfgs.E_INVALID_ARG
    assert create(S["gauss"], V["newton_schulz"], precision=1) == rbfgs.E_INVALID_ARG
    assert create(S["gauss"], V["mr"], precision=1) == rbfgs.E_INVALID_ARG
    assert create(4, V["fixed"]) == rbfgs.E_INVALID_ARG
    assert create(S["gauss"], 7) == rbfgs.E_INVALID_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_other_entry_points_validate_arguments():
    from paper_1602_01768_amd import rbfgs
    lib = rbfgs.load_library()
    buf = ctypes.c_void_p(256)
    it, rel = ctypes.c_int64(), ctypes.c_double()
    # partition draw: q must divide n, 1 <= q <= n, pointers set
    assert lib.rbfgs_sample_partition(buf, 10, 4, 1, 0, buf, None, None) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_sample_partition(buf, 8, 16, 1, 0, buf, None, None) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_sample_partition(None, 8, 4, 1, 0, buf, None, None) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_sample_partition(buf, 8, 4, 1, -1, buf, None, None) == rbfgs.E_INVALID_ARG
    # PCG and weights need a context
    assert lib.rbfgs_pcg(None, buf, 1, 1, buf, 1, 1, 1, 1e-8, 10, ctypes.byref(it), ctypes.byref(rel)) \
        == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_get_weights(None, buf) == rbfgs.E_INVALID_ARG
    # ridge Hessian: sizes, leading dimensions, finite scale and shift
    assert lib.rbfgs_ridge_hessian(buf, 1, 0, 4, 4, 1, 1.0, 0.0, buf, 1, 4, 1, None) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_ridge_hessian(buf, 1, 8, 4, 3, 1, 1.0, 0.0, buf, 1, 4, 1, None) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_ridge_hessian(buf, 1, 8, 4, 4, 1, float("nan"), 0.0, buf, 1, 4, 1, None) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_ridge_hessian(None, 1, 8, 4, 4, 1, 1.0, 0.0, buf, 1, 4, 1, None) == rbfgs.E_INVALID_ARG
    # the serving calls need a server
    assert lib.rbfgs_server_cancel(None, 0) == rbfgs.E_INVALID_ARG
    assert lib.rbfgs_server_stats(None, None) == rbfgs.E_INVALID_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_footprint_accounts_for_each_mode():
    """rbfgs_footprint is a dry run of the allocation code (no device memory is touched): it
    grows with n, the FP64 context holds more than the mixed one, and the partition weights,
    the importance Gram blocks and the AdaRBFGS probes add their buffers."""
    from paper_1602_01768_amd import rbfgs
    fp = rbfgs.rbfgs_footprint
    assert fp(4096, 64) < fp(8192, 64)
    assert fp(4096, 64, precision="mixed") < fp(4096, 64, precision="fp64")
    assert fp(4096, 64, sketch="partition") > fp(4096, 64, sketch="coord")
    assert fp(4096, 64, sketch="importance", variant="kaczmarz") > fp(4096, 64, sketch="coord", variant="kaczmarz")
    # the importance blocks of A A^T: r = n / q blocks of q_p x q_p FP64
    extra = fp(4096, 64, sketch="importance", variant="kaczmarz") - fp(4096, 64, sketch="coord", variant="kaczmarz")
    assert extra >= (4096 // 64) * 64 * 64 * 8
    assert fp(4096, 64, variant="adaptive") > 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_noalloc_ridge_hessian_validates_on_host():
    """The allocation-free entry point rejects bad arguments, and sizes beyond its fixed
    device array (8 (m_p n_p + n_p^2) + 256 bytes), before any device call."""
    from paper_1602_01768_amd import rbfgs
    lib = rbfgs.load_library()
    buf = ctypes.c_void_p(256)
    f = lib.rbfgs_ridge_hessian_noalloc
    assert f(buf, 1, 0, 4, 4, 1.0, 0.0, buf, 1, 4, None) == rbfgs.E_INVALID_ARG
    assert f(buf, 1, 8, 4, 3, 1.0, 0.0, buf, 1, 4, None) == rbfgs.E_INVALID_ARG
    assert f(buf, 1, 8, 4, 4, float("inf"), 0.0, buf, 1, 4, None) == rbfgs.E_INVALID_ARG
    assert f(None, 1, 8, 4, 4, 1.0, 0.0, buf, 1, 4, None) == rbfgs.E_INVALID_ARG
    assert f(buf, 1, 8, 4, 4, 1.0, 0.0, None, 1, 4, None) == rbfgs.E_INVALID_ARG
    assert f(buf, 1, 7153, 1024, 1024, 1.0, 0.0, buf, 0, 1024, None) == rbfgs.E_INVALID_ARG  # one row too many
    assert f(buf, 1, 100, 2944, 2944, 1.0, 0.0, buf, 0, 2944, None) == rbfgs.E_INVALID_ARG  # n_p^2 alone too big
    assert rbfgs.NOALLOC_SCRATCH_BYTES == 64 << 20
