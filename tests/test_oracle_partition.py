"""Pins of partition sampling with the probabilities of eq. (ihsih0) (CPU only).

What the mathematics fixes: for single coordinates the rate of fixed RBFGS under these
probabilities is exactly 1 - lambda_min(A) / Tr(A) (eq. rhoconv with W = A^-1) and the
one-step rate of AdaRBFGS exactly lambda_min(A X_k) / Tr(A X_k) (Theorem lem:9hs9hIKKK,
whose inequality is tight for q = 1); for blocks both are bounds.  The expected error
after one AdaRBFGS step, enumerated over all blocks with their probabilities, obeys the
theorem.  The Gram matrix of the whitened factor obeys L+^T A L+ = L^T A L - K K^T +
S~ (S~^T S~)^-1 S~^T with K = L^T Y R (the identity behind the O(nq) weight update).  The
draw's frequencies match the probabilities, and the estimator's mean is the residual.
"""
import numpy as np
import pytest

from oracle import partition as Pt, rbfgs as R, theory as T
from oracle.sketch import coord_matrix
from workloads import spectral_spd


def err_FA(X, A, Ainv):
    return R.error_FA(X, A, Ainv) ** 2


def test_blocks_and_rejection():
    parts = Pt.blocks(12, 4)
    assert [list(c) for c in parts] == [[0, 1, 2, 3], [4, 5, 6, 7], [8, 9, 10, 11]]
    with pytest.raises(ValueError):
        Pt.blocks(10, 4)


def test_weights_with_identity_factor_are_diagonal_block_sums():
    A, _ = spectral_spd(12, 1, 1.0, 50.0)
    w = Pt.block_weights_ada(np.eye(12), A, 3)
    assert np.allclose(w, np.diag(A).reshape(4, 3).sum(1), rtol=1e-14)
    assert np.allclose(Pt.block_weights_fixed(A, 3), w, rtol=1e-14)


def test_fixed_rate_single_coordinates_is_exact():
    """q = 1: E[Z] = A^2 / Tr(A), so rho = 1 - lambda_min(A) / Tr(A)."""
    n = 9
    A, _ = spectral_spd(n, 2, 1.0, 30.0)
    p = Pt.probabilities(Pt.block_weights_fixed(A, 1))
    EZ = T.expected_Z(A, [coord_matrix(C, n) for C in Pt.blocks(n, 1)], p)
    lam = np.linalg.eigvalsh(A)
    assert abs(T.rho_from_EZ(A, EZ) - (1.0 - lam[0] / lam.sum())) <= 1e-12
    # uniform probabilities give another rate: the pin sees the probabilities
    EZu = T.expected_Z(A, [coord_matrix(C, n) for C in Pt.blocks(n, 1)], [1.0 / n] * n)
    assert abs(T.rho_from_EZ(A, EZu) - T.rho_from_EZ(A, EZ)) > 1e-4


@pytest.mark.parametrize("n,q", [(12, 3), (16, 4)])
def test_fixed_rate_blocks_bounded(n, q):
    A, _ = spectral_spd(n, 3, 1.0, 30.0)
    p = Pt.probabilities(Pt.block_weights_fixed(A, q))
    rho = T.rho_from_EZ(A, T.expected_Z(A, [coord_matrix(C, n) for C in Pt.blocks(n, q)], p))
    lam = np.linalg.eigvalsh(A)
    assert 1.0 - q / n - 1e-12 <= rho <= 1.0 - lam[0] / lam.sum() + 1e-12


def ada_rate(L, A, q):
    """rho_k = lambda_min(A^-1/2 E[Z | X_k] A^-1/2) with S_i = L I_{:C_i} and eq. ihsih0."""
    n = A.shape[0]
    outs = [L @ coord_matrix(C, n) for C in Pt.blocks(n, q)]
    p = Pt.probabilities(Pt.block_weights_ada(L, A, q))
    return 1.0 - T.rho_from_EZ(A, T.expected_Z(A, outs, p))


def test_ada_rate_single_coordinates_is_exact():
    n = 8
    A, _ = spectral_spd(n, 4, 1.0, 40.0)
    L = Pt.run_ada(A, 1, 5, 6)
    AX = A @ L @ L.T
    ev = np.sort(np.linalg.eigvals(AX).real)
    assert abs(ada_rate(L, A, 1) - ev[0] / np.trace(AX)) <= 1e-12


@pytest.mark.parametrize("q,steps", [(2, 2), (4, 1), (3, 0)])
def test_ada_expected_error_obeys_theorem(q, steps):
    """Exact enumeration of E[||X+ - A^-1||^2_F(A) | X_k] over every block (X_k far from
    A^-1, so the comparison is not at rounding level)."""
    n = 12
    A, Ainv = spectral_spd(n, 5, 1.0, 40.0)
    L = Pt.run_ada(A, q, 9, steps)
    X = L @ L.T
    p = Pt.probabilities(Pt.block_weights_ada(L, A, q))
    expected = sum(pi * err_FA((Ln := R.ada_step(L, A, coord_matrix(C, n))) @ Ln.T, A, Ainv)
                   for pi, C in zip(p, Pt.blocks(n, q)))
    AX = A @ X
    ev = np.sort(np.linalg.eigvals(AX).real)
    bound = (1.0 - ev[0] / np.trace(AX)) * err_FA(X, A, Ainv)
    assert expected <= bound * (1 + 1e-10)
    assert ada_rate(L, A, q) >= ev[0] / np.trace(AX) - 1e-12


@pytest.mark.parametrize("kind", ["cols", "gauss"])
def test_whitened_gram_update_identity(kind):
    """L+^T A L+ = L^T A L - K K^T + S~ (S~^T S~)^-1 S~^T, K = L^T Y L_G^-T (eq. Cholimprov)."""
    n, q = 10, 3
    A, _ = spectral_spd(n, 6, 1.0, 20.0)
    L = R.run_ada(A, q, 2, "gauss", 3)
    if kind == "cols":
        St = coord_matrix(np.array([1, 4, 7]), n)
    else:
        St = np.random.default_rng(1).standard_normal((n, q))
    Y = A @ (L @ St)
    Lg = np.linalg.cholesky((L @ St).T @ Y)
    K = (L.T @ Y) @ np.linalg.inv(Lg).T
    Ln = R.ada_step(L, A, St)
    lhs = Ln.T @ A @ Ln
    rhs = L.T @ A @ L - K @ K.T + St @ np.linalg.solve(St.T @ St, St.T)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(lhs).max()


def test_draw_frequencies_match_probabilities():
    w = np.array([1.0, 3.0, 0.5, 2.5, 3.0])
    p = Pt.probabilities(w)
    N = 20000
    counts = np.bincount([Pt.draw(w, Pt.uniform(7, k)) for k in range(N)], minlength=5)
    chi2 = float(np.sum((counts - N * p) ** 2 / (N * p)))
    assert chi2 < 18.5  # 4 degrees of freedom, p-value 0.001


def test_draw_boundaries():
    w = np.array([1.0, 0.0, 1.0])
    assert Pt.draw(w, 1e-9) == 0 and Pt.draw(w, 0.5 - 1e-12) == 0 and Pt.draw(w, 0.5) == 2
    assert Pt.draw(w, 1.0 - 1e-16) == 2


@pytest.mark.parametrize("which", ["fixed", "ada"])
def test_estimator_mean_is_residual(which):
    """Sum over blocks of p_i * estimate_i equals the squared residual exactly."""
    n, q = 12, 4
    A, _ = spectral_spd(n, 8, 1.0, 20.0)
    if which == "fixed":
        X = Pt.run_fixed(A, q, 3, 4)
        p = Pt.probabilities(Pt.block_weights_fixed(A, q))
        est = [Pt.estimator_fixed(X, A, C, pi) for C, pi in zip(Pt.blocks(n, q), p)]
        ref = np.linalg.norm(np.eye(n) - X @ A) ** 2
    else:
        L = Pt.run_ada(A, q, 3, 4)
        p = Pt.probabilities(Pt.block_weights_ada(L, A, q))
        est = [Pt.estimator_ada(L, A, C, pi) for C, pi in zip(Pt.blocks(n, q), p)]
        ref = np.linalg.norm(np.eye(n) - L.T @ A @ L) ** 2
    assert abs(float(np.dot(p, est)) - ref) <= 1e-12 * ref


@pytest.mark.parametrize("which", ["fixed", "ada"])
def test_converges(which):
    n, q = 24, 4
    A, Ainv = spectral_spd(n, 10, 1.0, 50.0)
    if which == "fixed":
        X = Pt.run_fixed(A, q, 1, 3000)
    else:
        L = Pt.run_ada(A, q, 1, 60)
        X = L @ L.T
    assert np.linalg.norm(X - Ainv) <= 1e-6 * np.linalg.norm(Ainv)


# ---------------------------------------------------------------- importance (eq. discoptprob)
def kaczmarz_Z(A, S):
    """Z = A^T S (S^T A A^T S)^-1 S^T A, Alg. 1 with W = I."""
    P = A.T @ S
    return P @ np.linalg.solve(P.T @ P, P.T)


def gamma(A, outs, p):
    """gamma(p) = 1 - 1 / Tr(E[Z_p]^-1) (eq. 98h9s8h8s with W = I)."""
    EZ = sum(pi * kaczmarz_Z(A, S) for pi, S in zip(p, outs))
    return 1.0 - 1.0 / np.trace(np.linalg.inv(EZ))


def general_matrix(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) / np.sqrt(n) + 2.0 * np.eye(n) + np.diag(np.linspace(0.0, 3.0, n))


@pytest.mark.parametrize("q", [1, 2, 3])
def test_importance_with_exact_inverse_is_optimal(q):
    """With X = A^-1 the weights are those of eq. (discoptprob): gamma at them equals the
    closed form 1 - (sum_i w_i)^-2 of eq. (discoptrate) and is below gamma at every other p
    tried (uniform, the squared weights, random points of the simplex)."""
    n = 6
    A = general_matrix(n, q)
    Ainv = np.linalg.inv(A)
    outs = [coord_matrix(C, n) for C in Pt.blocks(n, q)]
    w = Pt.block_weights_importance(Ainv, A, q)
    p = Pt.probabilities(w)
    g = gamma(A, outs, p)
    assert abs(g - (1.0 - w.sum() ** -2)) <= 1e-12
    rng = np.random.default_rng(0)
    others = [np.full(len(outs), 1.0 / len(outs)), Pt.probabilities(w ** 2)]
    others += list(rng.dirichlet(np.ones(len(outs)), size=20))
    for po in others:
        assert gamma(A, outs, po) >= g - 1e-12


def test_importance_single_coordinates_is_product_of_norms():
    """q = 1: ||X e_i e_i^T A||_F = ||X e_i|| ||e_i^T A|| (the example of Sec. 7.2)."""
    n = 7
    A = general_matrix(n, 3)
    X = np.random.default_rng(4).standard_normal((n, n))
    w = Pt.block_weights_importance(X, A, 1)
    ref = np.linalg.norm(X, axis=0) * np.linalg.norm(A, axis=1)
    assert np.allclose(w, ref, rtol=1e-13)


def test_importance_estimator_mean_is_residual():
    n, q = 12, 3
    A = general_matrix(n, 5)
    X = Pt.run_kaczmarz_importance(A, q, 2, 5)
    p = Pt.probabilities(Pt.block_weights_importance(X, A, q))
    est = [Pt.estimator_rows(X, A, C, pi) for C, pi in zip(Pt.blocks(n, q), p)]
    ref = np.linalg.norm(np.eye(n) - A @ X) ** 2
    assert abs(float(np.dot(p, est)) - ref) <= 1e-12 * ref


def test_importance_kaczmarz_converges():
    """Not guaranteed by the theory (Sec. 7.2); on this well-conditioned matrix it converges."""
    n, q = 24, 4
    A = general_matrix(n, 6)
    X = Pt.run_kaczmarz_importance(A, q, 1, 1500)
    assert np.linalg.norm(np.eye(n) - A @ X) <= 1e-8 * np.sqrt(n)
