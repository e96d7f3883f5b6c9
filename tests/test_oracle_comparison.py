"""Pins of the oracle's comparison methods (Newton-Schulz, MR; Sec. 10), CPU only.

Each is checked against what the mathematics fixes: the power-method norm against the
library 2-norm, the Newton-Schulz residual recursion I - A X+ = (I - A X)^2, the MR step
length and starting scale as the minimisers of a scalar quadratic (found by fitting it
through three evaluations, not by the trace formulas), and convergence.
"""
import numpy as np
import pytest

from oracle import comparison as Cm
from workloads import spectral_spd


def quad_argmin(f):
    """Minimiser of the scalar quadratic f, from its values at -1, 0, 1."""
    a, b, c = np.polyfit([-1.0, 0.0, 1.0], [f(-1.0), f(0.0), f(1.0)], 2)
    return -b / (2 * a)


def test_power_norm_matches_two_norm():
    A, _ = spectral_spd(80, 3, 1.0, 50.0)
    assert abs(Cm.power_norm(A, 400) - np.linalg.norm(A, 2)) <= 1e-9 * np.linalg.norm(A, 2)


def test_ns_start_contracts():
    """rho(I - X_0 A) < 1 for X_0 = 0.99 A^T / rho^2(A) (Sec. 10)."""
    A, _ = spectral_spd(60, 4, 1.0, 1e3)
    ev = np.linalg.eigvals(np.eye(60) - Cm.ns_x0(A) @ A)
    assert np.max(np.abs(ev)) < 1.0


def test_ns_residual_squares():
    """I - A X_{k+1} = (I - A X_k)^2 for eq. (Newton-Schulz) when A X_k = X_k A."""
    n = 50
    A, _ = spectral_spd(n, 5, 1.0, 20.0)
    X = Cm.ns_x0(A)
    I = np.eye(n)
    for _ in range(4):
        R = I - A @ X
        X = Cm.ns_step(X, A)
        assert np.abs((I - A @ X) - R @ R).max() <= 1e-12 * max(1.0, np.abs(R).max())


def test_mr_alpha_minimises_residual():
    """alpha of eq. (MRiter) minimises ||I - A (X + alpha X R)||_F^2 (eq. MRdef)."""
    n = 40
    A, _ = spectral_spd(n, 6, 1.0, 30.0)
    X = Cm.mr_x0(A)
    I = np.eye(n)
    for _ in range(3):
        P = X @ (I - A @ X)
        a_fit = quad_argmin(lambda a: np.linalg.norm(I - A @ (X + a * P)) ** 2)
        assert abs(Cm.mr_alpha(X, A) - a_fit) <= 1e-8 * abs(a_fit)
        X = Cm.mr_step(X, A)


def test_mr_start_is_projected_identity():
    """(Tr A / Tr(A A^T)) minimises ||I - c A||_F over c."""
    A, _ = spectral_spd(30, 7, 1.0, 10.0)
    c_fit = quad_argmin(lambda c: np.linalg.norm(np.eye(30) - c * A) ** 2)
    assert abs(Cm.mr_x0(A)[0, 0] - c_fit) <= 1e-10 * c_fit


@pytest.mark.parametrize("method,iters", [("newton_schulz", 12), ("mr", 60)])
def test_converges(method, iters):
    n = 64
    A, _ = spectral_spd(n, 8, 1.0, 20.0)
    X0 = Cm.ns_x0(A) if method == "newton_schulz" else Cm.mr_x0(A)
    r0 = np.linalg.norm(np.eye(n) - A @ X0)
    X = Cm.run(method, A, iters)
    assert np.linalg.norm(np.eye(n) - A @ X) <= 1e-2 * r0
