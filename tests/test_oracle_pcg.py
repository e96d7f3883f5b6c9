"""Pins of the PCG oracle (CPU only): the library's CG, finite termination, one-step
convergence with the exact inverse, and the M-orthogonality of the residuals."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import pcg as P
from workloads import spectral_spd


def test_matches_library_cg():
    A, _ = spectral_spd(60, 1, 1.0, 100.0)
    b = np.random.default_rng(1).standard_normal(60)
    x, k, rel = P.pcg(A, b, tol=1e-12)
    ref, info = spla.cg(A, b, rtol=1e-12, atol=0.0, maxiter=1000)
    assert info == 0 and np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


def test_finite_termination():
    """In exact arithmetic CG ends after at most n steps; with a well-conditioned A the FP64
    residual after n steps is at rounding level."""
    A, Ainv = spectral_spd(12, 2, 1.0, 3.0)
    b = np.random.default_rng(2).standard_normal(12)
    x, k, rel = P.pcg(A, b, iters=12)
    assert np.abs(x - Ainv @ b).max() <= 1e-12 * np.abs(Ainv @ b).max()


def test_exact_inverse_preconditioner_converges_in_one_step():
    A, Ainv = spectral_spd(40, 3, 1.0, 1e4)
    b = np.random.default_rng(3).standard_normal(40)
    x, k, rel = P.pcg(A, b, M=Ainv, iters=1)
    assert rel <= 1e-10


def test_residuals_are_M_orthogonal():
    A, _ = spectral_spd(30, 4, 1.0, 50.0)
    Mh, _ = spectral_spd(30, 5, 0.5, 2.0)  # some SPD preconditioner
    b = np.random.default_rng(4).standard_normal(30)
    rs = []
    P.pcg(A, b, M=Mh, iters=6, record=lambda k, x, r: rs.append(r.copy()))
    for i in range(len(rs)):
        for j in range(i):
            num = abs(rs[i] @ Mh @ rs[j])
            assert num <= 1e-9 * np.sqrt((rs[i] @ Mh @ rs[i]) * (rs[j] @ Mh @ rs[j]))
