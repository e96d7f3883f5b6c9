"""Randomized block BFGS (RBFGS) and AdaRBFGS, plain FP64 on the CPU.

Fixed-sketch RBFGS, Sec. 8.7, eq. (qunac): with W = A^-1 in Alg. 3,

    X_{k+1} = S G^-1 S^T + (I - S G^-1 S^T A) X_k (I - A S G^-1 S^T),
    G = S^T A S.

`fixed_step_literal` evaluates that formula as printed (O(n^3), small n only).
`fixed_step` evaluates the same formula with every product taken through the
n x q factors (distributivity only): with P = S G^-1 S^T, U = S G^-1,
Y = A S, V = X_k Y and H = Y^T V = S^T A X_k A S,

    P A X_k = U V^T,   X_k A P = V U^T,   P A X_k A P = U H U^T,   P = U G U^T,

so X_{k+1} = X_k - U V^T - V U^T + U (G + H) U^T.  The two agree to rounding
(pinned by tests).

AdaRBFGS, Sec. 9.3, Alg. 4 and eq. (Cholimprov): X_k = L_k L_k^T and, with
S = L_k S~, G = S^T A S, R R^T = G^-1 and C (S~^T S~) C^T = I,

    L_{k+1} = L_k + S R (C S~^T - R^T S^T A L_k).

Reading used here (and by the GPU path): R = L_G^-T from the Cholesky factor
G = L_G L_G^T, C = L_M^-1 from S~^T S~ = L_M L_M^T.  The algorithm box writes
R_k = (S~^T A S~)^-1/2 where the derivation just above it (eq. Chol with S = L_k S~)
needs (S^T A S)^-1/2; the derivation is followed.  Any square roots with the
stated products give the same X_{k+1} (pinned by tests); L_{k+1} itself depends
on the choice, so both sides use the Cholesky one.

Iterations start from X_0 = I (L_0 = I), as in the experiments of Sec. 10.
"""
import numpy as np
import scipy.linalg as sla

from . import sketch as _sk


class NotSPDError(ArithmeticError):
    """G = S^T A S (or S~^T S~) has no Cholesky factor: A is not SPD or S is rank deficient."""


def chol_lower(M):
    """Lower Cholesky factor of the symmetric matrix M (lower triangle used)."""
    try:
        return np.linalg.cholesky(M)
    except np.linalg.LinAlgError as exc:
        raise NotSPDError(str(exc)) from exc


# ---------------------------------------------------------------- fixed sketch
def fixed_step_literal(X, A, S):
    """eq. (qunac) evaluated as printed, O(n^3)."""
    n = A.shape[0]
    G = S.T @ A @ S
    P = S @ np.linalg.solve(G, S.T)
    I = np.eye(n)
    return P + (I - P @ A) @ X @ (I - A @ P)


def fixed_step(X, A, S):
    """eq. (qunac) with products taken through the n x q factors, O(n^2 q)."""
    Y = A @ S                      # A S
    G = S.T @ Y                    # S^T A S
    Lg = chol_lower(G)
    U = sla.cho_solve((Lg, True), S.T).T      # S G^-1  (G symmetric)
    V = X @ Y                      # X_k A S
    H = Y.T @ V                    # S^T A X_k A S
    K = G + H
    Xn = X - U @ V.T - V @ U.T + U @ K @ U.T
    return 0.5 * (Xn + Xn.T)       # X_{k+1} is symmetric (eq. NFsym constraint)


def estimator(X, A, S, kind):
    """Unbiased estimate of ||I - X A||_F^2 from the step's own products.

    S - X A S = (I - X A) S.  For S with i.i.d. N(0,1) entries E[S S^T] = q I, so
    E ||(I - XA) S||_F^2 = q ||I - XA||_F^2; for q coordinates drawn uniformly
    without replacement E = (q / n) ||I - XA||_F^2.  (||I - XA||_F = ||I - AX||_F
    for symmetric A and X.)
    """
    n, q = S.shape
    r2 = float(np.sum((S - X @ (A @ S)) ** 2))
    return r2 / q if kind == "gauss" else r2 * n / q


def first_step_entries(A, S, rows, cols, block=4096):
    """Entries (rows[t], cols[t]) of X_1 = eq. (qunac) applied to X_0 = I, for n too large to
    form n x n matrices.  With P = S G^-1 S^T, X_1 = P + (I - P A)(I - A P), and with Y = A S:
        X_1[i, j] = delta_ij + S_i G^-1 S_j^T - S_i G^-1 Y_j^T - Y_i G^-1 S_j^T
                    + S_i G^-1 (Y^T Y) G^-1 S_j^T,
    where S_i is row i of S.  A is promoted to FP64 in blocks of `block` rows to form Y."""
    n = A.shape[0]
    S = np.asarray(S, dtype=np.float64)
    Y = np.empty_like(S)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        Y[r0:r1] = np.asarray(A[r0:r1], dtype=np.float64) @ S
    G = S.T @ Y
    Lg = chol_lower(G)
    Gi = sla.cho_solve((Lg, True), np.eye(G.shape[0]))
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    Si, Sj, Yi, Yj = S[rows], S[cols], Y[rows], Y[cols]
    SiG, YiG = Si @ Gi, Yi @ Gi
    K = Gi @ (Y.T @ Y) @ Gi
    return ((rows == cols).astype(np.float64) + np.einsum("tk,tk->t", SiG, Sj) - np.einsum("tk,tk->t", SiG, Yj)
            - np.einsum("tk,tk->t", YiG, Sj) + np.einsum("tk,tk->t", Si @ K, Sj))


# ------------------------------------------------------------------- AdaRBFGS
def ada_step(L, A, St):
    """One AdaRBFGS factor update, eq. (Cholimprov), Cholesky square roots."""
    S = L @ St                                   # S = L_k S~
    Y = A @ S
    G = S.T @ Y                                  # S^T A S
    Lg = chol_lower(G)
    R = sla.solve_triangular(Lg, np.eye(G.shape[0]), lower=True).T   # L_G^-T
    Lm = chol_lower(St.T @ St)
    C = sla.solve_triangular(Lm, np.eye(Lm.shape[0]), lower=True)    # L_M^-1
    return L + S @ R @ (C @ St.T - R.T @ (Y.T @ L))


def ada_step_sqrt(L, A, St):
    """Same update with symmetric inverse square roots (eigendecomposition).

    Only used to pin that X_{k+1} = L_{k+1} L_{k+1}^T does not depend on the
    choice of square roots.
    """
    S = L @ St
    Y = A @ S
    G = S.T @ Y
    w, Q = np.linalg.eigh(G)
    R = Q @ np.diag(w ** -0.5) @ Q.T
    w2, Q2 = np.linalg.eigh(St.T @ St)
    C = Q2 @ np.diag(w2 ** -0.5) @ Q2.T
    return L + S @ R @ (C @ St.T - R.T @ (Y.T @ L))


def ada_estimator(L, A, St, kind):
    """Unbiased estimate of ||I - L^T A L||_F^2 (same argument as `estimator`
    applied to the symmetric matrix L^T A L, which is similar to A X)."""
    n, q = St.shape
    r2 = float(np.sum((St - L.T @ (A @ (L @ St))) ** 2))
    return r2 / q if kind == "gauss" else r2 * n / q


# ------------------------------------------------------------------ residuals
def residual_fro(A, X):
    """||I - A X||_F in FP64."""
    return float(np.linalg.norm(np.eye(A.shape[0]) - A @ X))


def error_FA(X, A, Ainv):
    """||X - A^-1||_{F(A)} = ||A^1/2 (X - A^-1) A^1/2||_F (eq. 98y988ff, W = A^-1)."""
    E = X - Ainv
    return float(np.sqrt(max(np.trace(E @ A @ E @ A), 0.0)))


# -------------------------------------------------------------------- drivers
def run_fixed(A, q, seed, kind, iters, X0=None, record=None, literal=False):
    """`iters` fixed-sketch RBFGS steps from X0 (default I) on the seeded stream.

    record(k, X) is called after every step when given.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    X = np.eye(n) if X0 is None else np.array(X0, dtype=np.float64)
    step = fixed_step_literal if literal else fixed_step
    for k in range(iters):
        S = _sk.sketch(seed, k, n, q, kind)
        X = step(X, A, S)
        if record is not None:
            record(k, X)
    return X


def run_ada(A, q, seed, kind, iters, L0=None, record=None):
    """`iters` AdaRBFGS steps from L0 (default I); returns L."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.eye(n) if L0 is None else np.array(L0, dtype=np.float64)
    for k in range(iters):
        St = _sk.sketch(seed, k, n, q, kind)
        L = ada_step(L, A, St)
        if record is not None:
            record(k, L)
    return L
