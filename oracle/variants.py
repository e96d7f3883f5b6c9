"""Other instances of the sketch-and-project family, plain FP64 on the CPU.

All three take one step of Alg. 1 (row variant) or Alg. 3 (symmetric variant) for a
particular weight W, each drawing a fresh sketch S per iteration:

* Simultaneous randomized Kaczmarz, Sec. 8.2, eq. (badbroyadj): Alg. 1 with W = I,
  for any invertible A,
      X+ = X + A^T S (S^T A A^T S)^-1 S^T (I - A X).
* Approximate inverse preconditioning (AIP), Sec. 8.6, eq. (BFGSas): Alg. 1 with
  W = A^-1, A symmetric positive definite,
      X+ = X + S (S^T A S)^-1 S^T (I - A X).
* Randomized Powell-symmetric-Broyden (PSB), Sec. 8.4: Alg. 3 with W = I, A
  symmetric.  The printed eq. (PSB) has garbled transposes; this module follows
  the general closed form eq. (Xupdatesym) with W = I and Lambda = (S^T A^2 S)^-1:
      X+ = X - (X A - I) S Lambda S^T A + A S Lambda S^T (A X - I)(A S Lambda S^T A - I).

`*_literal` evaluate the printed formula (O(n^3), small n only; the Kaczmarz and
AIP forms through Alg. 1's Lambda = S (S^T A W A^T S)^-1 S^T with W explicit).
The factored forms take every product through n x q factors (distributivity only):

* Kaczmarz / AIP, with P = A^T S (Kaczmarz) or P = A S (AIP, A = A^T), and
  U = P G^-1 with G = P^T P (Kaczmarz) or U = S G^-1 with G = S^T P (AIP):
      S^T (I - A X) = S^T - P^T X,   X+ = X + U (S^T - P^T X).
* PSB, with Y = A S, G = Y^T Y = S^T A^2 S, U = Y G^-1, V = X Y, R = V - S and
  H' = R^T Y = Y^T V - S^T Y (symmetric for symmetric A and X):
      X+ = X - R U^T - U R^T + U H' U^T = X - (U W'^T + W' U^T),  W' = R - U H'/2,
  the same symmetric rank-2q shape as fixed RBFGS (which has U = S G^-1, G = S^T Y).

The residual sketch of the two row variants is S^T (I - A X) = S^T - P^T X,
which the step forms anyway; with Gaussian S its squared norm over q estimates
||I - A X||_F^2 without bias (E[S S^T] = q I).

Iterations start from X_0 = I.
"""
import numpy as np
import scipy.linalg as sla

from . import sketch as _sk
from .rbfgs import chol_lower


# ------------------------------------------------------------ literal forms
def alg1_step_literal(X, A, S, W):
    """Alg. 1 (row variant) as printed: Lambda = S (S^T A W A^T S)^-1 S^T,
    X+ = X + W A^T Lambda (I - A X)."""
    n = A.shape[0]
    Lam = S @ np.linalg.solve(S.T @ A @ W @ A.T @ S, S.T)
    return X + W @ A.T @ Lam @ (np.eye(n) - A @ X)


def kaczmarz_step_literal(X, A, S):
    """eq. (badbroyadj): Alg. 1 with W = I."""
    return alg1_step_literal(X, A, S, np.eye(A.shape[0]))


def aip_step_literal(X, A, S):
    """eq. (BFGSas): Alg. 1 with W = A^-1 (A SPD)."""
    return alg1_step_literal(X, A, S, np.linalg.inv(A))


def psb_step_literal(X, A, S):
    """eq. (Xupdatesym) with W = I: the randomized PSB step (A symmetric)."""
    n = A.shape[0]
    I = np.eye(n)
    AS = A @ S
    Lam = np.linalg.inv(AS.T @ AS)                    # (S^T A W A S)^-1 with W = I
    return X - (X @ A - I) @ S @ Lam @ S.T @ A + AS @ Lam @ S.T @ (A @ X - I) @ (AS @ Lam @ S.T @ A - I)


# ------------------------------------------------------------ factored forms
def kaczmarz_step(X, A, S):
    """eq. (badbroyadj) through n x q factors: P = A^T S, G = P^T P, U = P G^-1."""
    P = A.T @ S
    G = P.T @ P
    U = sla.cho_solve((chol_lower(G), True), P.T).T
    return X + U @ (S.T - P.T @ X)


def aip_step(X, A, S):
    """eq. (BFGSas) through n x q factors: P = A S, G = S^T P, U = S G^-1."""
    P = A @ S
    G = S.T @ P
    U = sla.cho_solve((chol_lower(G), True), S.T).T
    return X + U @ (S.T - P.T @ X)


def psb_step(X, A, S):
    """Randomized PSB through n x q factors (see the module notes)."""
    Y = A @ S
    G = Y.T @ Y                                       # S^T A^2 S
    U = sla.cho_solve((chol_lower(G), True), Y.T).T   # Y G^-1
    V = X @ Y
    R = V - S                                         # (X A - I) S
    Hp = Y.T @ V - S.T @ Y                            # R^T Y
    Wp = R - 0.5 * U @ Hp
    Xn = X - U @ Wp.T - Wp @ U.T
    return 0.5 * (Xn + Xn.T)                          # symmetric by construction (eq. NFsym)


STEPS = {"kaczmarz": kaczmarz_step, "aip": aip_step, "psb": psb_step}
STEPS_LITERAL = {"kaczmarz": kaczmarz_step_literal, "aip": aip_step_literal, "psb": psb_step_literal}


def row_estimator(X, A, S, kind):
    """Unbiased estimate of ||I - A X||_F^2 from S^T (I - A X) (Kaczmarz, AIP).

    For S with i.i.d. N(0,1) entries E[S S^T] = q I, so E ||S^T M||_F^2 = q ||M||_F^2;
    for q coordinates drawn uniformly without replacement E = (q / n) ||M||_F^2.
    """
    n, q = S.shape
    r2 = float(np.sum((S.T - S.T @ A @ X) ** 2))
    return r2 / q if kind == "gauss" else r2 * n / q


def run(variant, A, q, seed, kind, iters, X0=None, record=None, literal=False):
    """`iters` steps of `variant` ('kaczmarz', 'aip', 'psb') from X0 (default I) on
    the seeded sketch stream (the same stream as fixed RBFGS)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    X = np.eye(n) if X0 is None else np.array(X0, dtype=np.float64)
    step = (STEPS_LITERAL if literal else STEPS)[variant]
    for k in range(iters):
        S = _sk.sketch(seed, k, n, q, kind)
        X = step(X, A, S)
        if record is not None:
            record(k, X)
    return X
