"""GPU parity of the ridge Hessian step (eq. ridgeMatrix) through the C ABI."""
import numpy as np
import pytest

from oracle import ridge
from workloads import ridge_data

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n", [(1, 1), (7, 5), (517, 300), (300, 517), (2048, 1024)])
@pytest.mark.parametrize("b_dtype", [np.float32, np.float64])
@pytest.mark.parametrize("on_device", [False, True])
def test_matches_oracle_fp64_out(lib, m, n, b_dtype, on_device):
    import torch
    B = np.random.default_rng(m * n).standard_normal((m, n)).astype(b_dtype)
    Bin = torch.from_numpy(B).cuda() if on_device else B
    A = lib.rbfgs_ridge_hessian(Bin, 1.0 / m, 1e-2, dtype=lib.F64).cpu().numpy()
    ref = ridge.ridge_hessian(B, 1.0 / m, 1e-2)
    assert np.abs(A - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.array_equal(A, A.T)


def test_fp32_output_is_rounded_fp64(lib):
    """The FP32 result equals the FP64 one rounded (to within one ulp where the FP64
    values differ from the oracle's in the last bits)."""
    B = ridge_data(384, 7, m=768)
    A32 = lib.rbfgs_ridge_hessian(B, 1.0 / 768, 1e-2, dtype=lib.F32).cpu().numpy()
    ref = ridge.ridge_hessian(B, 1.0 / 768, 1e-2).astype(np.float32)
    ulp = np.spacing(np.abs(ref))
    assert np.all(np.abs(A32 - ref) <= ulp)


def test_invalid_arguments(lib):
    with pytest.raises(lib.RbfgsError) as ei:
        lib.rbfgs_ridge_hessian(np.ones((4, 3)), float("nan"), 0.0)
    assert ei.value.status == lib.E_INVALID_ARG
