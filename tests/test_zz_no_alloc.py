"""The allocation-free ridge-Hessian entry point (work buffers in the library's fixed device
array) against the allocating one, through the C ABI: two calls in a row, the second with a
smaller input (the array keeps the first call's contents, which must not leak into the
second), FP32 and FP64 data and outputs, and sizes beyond the array rejected."""
import numpy as np
import pytest

from oracle import ridge

pytestmark = pytest.mark.gpu


def data(m, n, dtype, seed):
    return np.random.default_rng(seed).standard_normal((m, n)).astype(dtype)


@pytest.mark.parametrize("b_dtype,out_dtype", [(np.float32, np.float32), (np.float64, np.float64),
                                               (np.float32, np.float64)])
def test_matches_allocating_entry_point(lib, b_dtype, out_dtype):
    import torch
    tout = torch.float32 if out_dtype == np.float32 else torch.float64
    for m, n, seed in ((1500, 1000, 1), (37, 29, 2)):  # second call smaller
        B = data(m, n, b_dtype, seed)
        Bd = torch.from_numpy(B).cuda()
        out = torch.full((n, n), float("nan"), dtype=tout, device="cuda")
        print(f"noalloc ridge m={m} n={n} {np.dtype(b_dtype).name}->{np.dtype(out_dtype).name}", flush=True)
        lib.rbfgs_ridge_hessian_noalloc(Bd, 1.0 / m, 1e-2, out)
        ref = lib.rbfgs_ridge_hessian(Bd, 1.0 / m, 1e-2, dtype=lib.F32 if out_dtype == np.float32 else lib.F64)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy())
        if out_dtype == np.float64:
            orc = ridge.ridge_hessian(B, 1.0 / m, 1e-2)
            assert np.abs(got - orc).max() <= 1e-13 * np.abs(orc).max()


def test_limit_rejected(lib):
    import torch
    n = 1024
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    B_ok = torch.zeros((7152, n), dtype=torch.float32, device="cuda")
    lib.rbfgs_ridge_hessian_noalloc(B_ok, 1.0, 0.0, out)  # the largest m that fits at n = 1024
    torch.cuda.synchronize()
    assert torch.all(out == 0)
    B_big = torch.zeros((7153, n), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.RbfgsError) as ei:
        lib.rbfgs_ridge_hessian_noalloc(B_big, 1.0, 0.0, out)
    assert ei.value.status == lib.E_INVALID_ARG
