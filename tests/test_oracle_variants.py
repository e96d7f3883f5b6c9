"""Pins of the oracle's other sketch-and-project instances (CPU only).

Simultaneous randomized Kaczmarz (eq. badbroyadj), AIP (eq. BFGSas) and randomized
PSB (eq. Xupdatesym with W = I) are checked against the projection they are defined
by (eq. NF / eq. NFsym, solved densely as a KKT system), against the printed
formulas, and against properties the paper states: one-step convergence with a
full-rank square sketch (Sec. 8.1), A^-1 as a fixed point, the sketched equation
holding after a step, an unbiased residual estimator, and convergence.
"""
import numpy as np
import pytest

from oracle import sketch as sk, theory as T, variants as V
from workloads import spectral_spd

VARIANTS = ["kaczmarz", "aip", "psb"]


def problem(variant, n, seed):
    """A matrix each variant is defined for: general invertible (Kaczmarz), SPD
    (AIP), symmetric indefinite (PSB)."""
    rng = np.random.default_rng(seed)
    if variant == "kaczmarz":
        A = rng.standard_normal((n, n)) + 2.0 * np.sqrt(n) * np.eye(n)
    elif variant == "aip":
        A = spectral_spd(n, seed, 1.0, 20.0)[0]
    else:
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = np.linspace(1.0, 4.0, n) * np.where(np.arange(n) % 3 == 0, -1.0, 1.0)
        A = (Q * lam) @ Q.T
        A = 0.5 * (A + A.T)
    return A


def weight_inverse(variant, A):
    """W^-1 of the weighted norm the variant projects in."""
    return A if variant == "aip" else np.eye(A.shape[0])


def start(variant, n, seed):
    rng = np.random.default_rng(seed + 100)
    X = rng.standard_normal((n, n)) / n
    return X + X.T if variant == "psb" else X


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n,q", [(5, 1), (6, 2), (7, 3), (6, 5)])
def test_step_is_the_weighted_projection(variant, n, q):
    """The factored step equals argmin ||X - X_k||_{F(W^-1)} s.t. S^T A X = S^T
    (and X = X^T for PSB), solved as a dense KKT system."""
    A = problem(variant, n, 3 * n + q)
    X = start(variant, n, n + q)
    S = np.random.default_rng(n * q).standard_normal((n, q))
    want = T.projection_kkt_weighted(X, A, S, weight_inverse(variant, A), variant == "psb")
    got = V.STEPS[variant](X, A, S)
    assert np.abs(got - want).max() <= 1e-10 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind", ["gauss", "cols"])
def test_factored_equals_literal_along_trajectory(variant, kind):
    """The n x q form and the printed O(n^3) formula agree to rounding over
    several steps of the seeded stream."""
    n, q = 24, 4
    A = problem(variant, n, 11)
    Xf = V.run(variant, A, q, 5, kind, 6)
    Xl = V.run(variant, A, q, 5, kind, 6, literal=True)
    assert np.abs(Xf - Xl).max() <= 1e-9 * max(1.0, np.abs(Xl).max())


@pytest.mark.parametrize("variant", VARIANTS)
def test_one_step_with_square_sketch(variant):
    """S = I (q = n): the sketched equation is AX = I, so X_1 = A^-1 (Sec. 8.1)."""
    n = 9
    A = problem(variant, n, 4)
    X1 = V.STEPS[variant](start(variant, n, 4), A, np.eye(n))
    assert np.abs(X1 - np.linalg.inv(A)).max() <= 1e-10 * np.abs(np.linalg.inv(A)).max()


@pytest.mark.parametrize("variant", VARIANTS)
def test_inverse_is_fixed_point_and_constraint_holds(variant):
    n, q = 12, 3
    A = problem(variant, n, 6)
    Ainv = np.linalg.inv(A)
    S = sk.gaussian_sketch(1, 0, n, q)
    assert np.abs(V.STEPS[variant](Ainv, A, S) - Ainv).max() <= 1e-11 * np.abs(Ainv).max()
    X1 = V.STEPS[variant](start(variant, n, 6), A, S)
    assert np.abs(S.T @ A @ X1 - S.T).max() <= 1e-10 * np.abs(S).max()
    if variant == "psb":
        assert np.array_equal(X1, X1.T)


@pytest.mark.parametrize("variant", ["kaczmarz", "aip"])
def test_row_estimator_unbiased_exact_for_coordinates(variant):
    """Averaging over all q-subsets gives ||I - A X||_F^2 exactly."""
    n = 6
    A = problem(variant, n, 8)
    X = start(variant, n, 8)
    truth = np.linalg.norm(np.eye(n) - A @ X) ** 2
    for q in (1, 2, 3):
        outs, probs = T.uniform_subsets(n, q)
        avg = sum(p * V.row_estimator(X, A, S, "cols") for S, p in zip(outs, probs))
        assert abs(avg - truth) <= 1e-12 * truth


def test_row_estimator_unbiased_gaussian():
    n, q = 40, 4
    A = problem("kaczmarz", n, 9)
    X = start("kaczmarz", n, 9)
    truth = np.linalg.norm(np.eye(n) - A @ X) ** 2
    ests = [V.row_estimator(X, A, sk.gaussian_sketch(s, 0, n, q), "gauss") for s in range(400)]
    assert abs(np.mean(ests) - truth) <= 0.05 * truth


def test_kaczmarz_expected_error_one_step_exact():
    """For S drawn uniformly among q-subsets of coordinates, E_{k+1} = (I - Z) E_k with
    the projection Z = A^T S (S^T A A^T S)^-1 S^T A, so the mean of ||E_{k+1}||_F^2
    over all subsets equals tr(E_k^T (I - E[Z]) E_k) (Sec. 6, eq. for the error)."""
    n, q = 6, 2
    A = problem("kaczmarz", n, 12)
    Ainv = np.linalg.inv(A)
    X = start("kaczmarz", n, 12)
    E = X - Ainv
    outs, probs = T.uniform_subsets(n, q)
    mean_sq = sum(p * np.linalg.norm(V.kaczmarz_step(X, A, S) - Ainv) ** 2 for S, p in zip(outs, probs))
    EZ = sum(p * (A.T @ S @ np.linalg.solve(S.T @ A @ A.T @ S, S.T @ A)) for S, p in zip(outs, probs))
    assert abs(mean_sq - np.trace(E.T @ (np.eye(n) - EZ) @ E)) <= 1e-12 * mean_sq


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind", ["gauss", "cols"])
def test_converges(variant, kind):
    n, q = 32, 8
    A = problem(variant, n, 21)
    r0 = np.linalg.norm(np.eye(n) - A) / np.sqrt(n)
    X = V.run(variant, A, q, 9, kind, 300)
    r = np.linalg.norm(np.eye(n) - A @ X) / np.sqrt(n)
    assert r <= 1e-3 * r0
