"""Pins of the ridge Hessian oracle (eq. ridgeMatrix), CPU only."""
import numpy as np

from oracle import ridge


def test_matches_entrywise_sums():
    """Each entry against its definition as a sum over the m data rows (plain loops)."""
    rng = np.random.default_rng(1)
    m, n, scale, lam = 7, 5, 1.0 / 7, 0.3
    B = rng.standard_normal((m, n))
    H = ridge.ridge_hessian(B, scale, lam)
    for i in range(n):
        for j in range(n):
            s = sum(float(B[r, i]) * float(B[r, j]) for r in range(m))
            assert abs(H[i, j] - (scale * s + (lam if i == j else 0.0))) <= 1e-13


def test_is_the_hessian_of_the_objective():
    """The objective is quadratic, so differences of its gradient along e_j are exactly
    H e_j (up to rounding): a check through the objective, not the formula."""
    rng = np.random.default_rng(2)
    m, n, scale, lam = 40, 12, 1.0 / 40, 1e-2
    B = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    x = rng.standard_normal(n)
    H = ridge.ridge_hessian(B, scale, lam)
    g0 = ridge.ridge_objective_grad(B, b, lam, x, scale)
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        col = ridge.ridge_objective_grad(B, b, lam, x + e, scale) - g0
        assert np.abs(col - H[:, j]).max() <= 1e-12 * max(1.0, np.abs(H).max())


def test_symmetric_and_bounded_below_by_lambda():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((9, 20))  # rank 9 < n: the smallest eigenvalue is lam
    H = ridge.ridge_hessian(B, 0.5, 0.25)
    assert np.array_equal(H, H.T) or np.abs(H - H.T).max() <= 1e-15
    ev = np.linalg.eigvalsh(H)
    assert abs(ev[0] - 0.25) <= 1e-12 and ev[-1] > 0.25
