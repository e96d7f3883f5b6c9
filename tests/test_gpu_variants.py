"""GPU parity of the other sketch-and-project instances (PSB, AIP, simultaneous
randomized Kaczmarz) through the C ABI against the FP64 oracle.

Same bars as the fixed method: relative Frobenius error of X <= 1e-10 in FP64 mode
and <= 1e-4 in mixed mode (A given in FP32 so that both sides invert the same
matrix) at a fixed iteration count.
"""
import math

import numpy as np
import pytest

from oracle import sketch as sk, variants as V
from workloads import spectral_spd

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4
VARIANTS = ["psb", "aip", "kaczmarz"]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def matrix(variant, n, seed, dtype=np.float64):
    """General invertible (Kaczmarz: I-dominated, not symmetric), SPD (AIP) or
    symmetric indefinite (PSB) test matrices."""
    rng = np.random.default_rng(seed)
    if variant == "kaczmarz":
        A = rng.standard_normal((n, n)) / math.sqrt(n) + 2.5 * np.eye(n)
    elif variant == "aip":
        A = spectral_spd(n, seed, 1.0, 100.0)[0]
    else:
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = np.linspace(1.0, 4.0, n) * np.where(np.arange(n) % 3 == 0, -1.0, 1.0)
        A = (Q * lam) @ Q.T
        A = 0.5 * (A + A.T)
    return np.ascontiguousarray(A.astype(dtype))


def gpu_x(lib, A, q, seed, kind, variant, precision, steps):
    import torch
    with lib.Solver(A, q, seed, sketch=kind, variant=variant, precision=precision) as s:
        s.step(steps)
        s.sync()
        X = s.x().cpu().numpy()
    torch.cuda.synchronize()
    return X


def oracle_x(A, q, seed, kind, variant, steps):
    return V.run(variant, np.asarray(A, np.float64), q, seed, "cols" if kind == "coord" else kind, steps)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind", ["gauss", "coord"])
@pytest.mark.parametrize("n,q,steps", [(1, 1, 2), (37, 5, 20), (300, 17, 30), (257, 130, 6)])
def test_fp64_parity(lib, variant, kind, n, q, steps):
    A = matrix(variant, n, n + q)
    assert rel(gpu_x(lib, A, q, 5, kind, variant, "fp64", steps), oracle_x(A, q, 5, kind, variant, steps)) <= FP64_TOL


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind", ["gauss", "coord"])
def test_mixed_parity(lib, variant, kind):
    n, q, steps = 520, 40, 60
    A = matrix(variant, n, 3, np.float32)
    assert rel(gpu_x(lib, A, q, 2, kind, variant, "mixed", steps), oracle_x(A, q, 2, kind, variant, steps)) <= MIXED_TOL


@pytest.mark.parametrize("variant", VARIANTS)
def test_mixed_parity_tiles(lib, variant):
    """Several 128 x 128 tiles of the update and split-K chunks of the products."""
    n, q, steps = 1024, 64, 12
    A = matrix(variant, n, 7, np.float32)
    assert rel(gpu_x(lib, A, q, 4, "gauss", variant, "mixed", steps), oracle_x(A, q, 4, "gauss", variant, steps)) <= MIXED_TOL


@pytest.mark.parametrize("variant", VARIANTS)
def test_one_step_exact_when_q_equals_n(lib, variant):
    """A full-rank square sketch makes the sketched equation A X = I (Sec. 8.1)."""
    A = matrix(variant, 48, 2)
    assert rel(gpu_x(lib, A, 48, 1, "gauss", variant, "fp64", 1), np.linalg.inv(A)) <= 1e-9


@pytest.mark.parametrize("variant", VARIANTS)
def test_residual_matches_oracle(lib, variant):
    """The exact residual ||I - A X||_F, in particular for the nonsymmetric iterates."""
    A = matrix(variant, 200, 9)
    with lib.Solver(A, 12, 3, variant=variant) as s:
        s.step(10)
        r = s.residual()
    Xo = oracle_x(A, 12, 3, "gauss", variant, 10)
    assert abs(r - np.linalg.norm(np.eye(200) - A @ Xo)) <= 1e-9 * r


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-4)])
@pytest.mark.parametrize("variant", ["aip", "kaczmarz"])
def test_row_estimator_matches_oracle(lib, variant, precision, tol):
    """The estimator of the row variants is ||S^T (I - A X_k)||^2 / q, taken from the
    step's own product X^T P (fused into its reduction in mixed mode)."""
    n, q = 512, 16
    A = matrix(variant, n, 4, np.float32)
    X = oracle_x(A, q, 8, "gauss", variant, 4)
    S = sk.gaussian_sketch(8, 4, n, q)
    with lib.Solver(A, q, 8, variant=variant, precision=precision) as s:
        s.step(5)
        est = s.estimate()
    ref = V.row_estimator(X, np.asarray(A, np.float64), S, "gauss")
    assert abs(est - ref) <= tol * ref


@pytest.mark.parametrize("variant", VARIANTS)
def test_invert_converges(lib, variant):
    n = 96
    A = matrix(variant, n, 5)
    with lib.Solver(A, 24, 1, variant=variant, check_every=4) as s:
        ok, iters, resid = s.invert(tol=1e-8, max_iters=3000)
        assert ok and resid <= 1e-8
        X = s.x().cpu().numpy()
    assert np.linalg.norm(np.eye(n) - A @ X) / math.sqrt(n) <= 1e-8


def test_symmetry_required_except_for_kaczmarz(lib):
    A = matrix("kaczmarz", 32, 1)
    for variant in ("fixed", "adaptive", "psb", "aip"):
        with pytest.raises(lib.RbfgsError) as ei:
            lib.Solver(A, 4, 1, variant=variant)
        assert ei.value.status == lib.E_INVALID_ARG
    with lib.Solver(A, 4, 1, variant="kaczmarz") as s:
        s.step(2)
        s.sync()
