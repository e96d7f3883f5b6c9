"""GPU parity of the comparison methods of Sec. 10 (Newton-Schulz, MR) through the C ABI
against the FP64 oracle, including their starting points."""
import math

import numpy as np
import pytest

from oracle import comparison as Cm
from workloads import spectral_spd

pytestmark = pytest.mark.gpu

METHODS = ["newton_schulz", "mr"]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rand_spd(n, seed):
    """A = M^T M with M uniform on [0, 1) (a matrix built from rand, as in Experiment 1)."""
    M = np.random.default_rng(seed).random((n, n))
    return M.T @ M


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("n", [1, 37, 257, 300])
def test_start_matches_oracle(lib, method, n):
    A, _ = spectral_spd(n, n, 1.0, 100.0)
    with lib.Solver(A, 1, 1, variant=method) as s:
        X0 = s.x().cpu().numpy()
    ref = Cm.ns_x0(A) if method == "newton_schulz" else Cm.mr_x0(A)
    assert rel(X0, ref) <= 1e-12


@pytest.mark.parametrize("method,iters", [("newton_schulz", 8), ("mr", 12)])
@pytest.mark.parametrize("n", [37, 257, 300])
def test_fp64_parity(lib, method, iters, n):
    A, _ = spectral_spd(n, 2 * n, 1.0, 100.0)
    with lib.Solver(A, 1, 1, variant=method) as s:
        s.step(iters)
        X = s.x().cpu().numpy()
    assert rel(X, Cm.run(method, A, iters)) <= 1e-10


@pytest.mark.parametrize("method", METHODS)
def test_parity_rand_matrix(lib, method):
    """The ill-conditioned rand-based matrices of Experiment 1 (kappa ~ 1e8 at n = 500)."""
    A = rand_spd(500, 4)
    iters = 20 if method == "newton_schulz" else 8
    with lib.Solver(A, 1, 1, variant=method) as s:
        s.step(iters)
        X = s.x().cpu().numpy()
    assert rel(X, Cm.run(method, A, iters)) <= 1e-9


@pytest.mark.parametrize("method", METHODS)
def test_estimate_is_residual_of_step_start(lib, method):
    """The estimator is the exact ||I - A X_k||_F^2 of the iterate the last step started from."""
    A, _ = spectral_spd(128, 5, 1.0, 20.0)
    Xk = Cm.run(method, A, 3)
    with lib.Solver(A, 1, 1, variant=method) as s:
        s.step(4)
        est = s.estimate()
    ref = np.linalg.norm(np.eye(128) - A @ Xk) ** 2
    assert abs(est - ref) <= 1e-9 * ref


@pytest.mark.parametrize("method", METHODS)
def test_invert_converges(lib, method):
    n = 96
    A, _ = spectral_spd(n, 6, 1.0, 20.0)
    with lib.Solver(A, 1, 1, variant=method, check_every=1) as s:
        ok, iters, resid = s.invert(tol=1e-8, max_iters=500)
        assert ok and resid <= 1e-8
        X = s.x().cpu().numpy()
    assert np.linalg.norm(np.eye(n) - A @ X) / math.sqrt(n) <= 1e-8


@pytest.mark.parametrize("method", METHODS)
def test_mixed_precision_rejected(lib, method):
    A, _ = spectral_spd(64, 1)
    with pytest.raises(lib.RbfgsError) as ei:
        lib.Solver(A.astype(np.float32), 1, 1, variant=method, precision="mixed")
    assert ei.value.status == lib.E_INVALID_ARG
