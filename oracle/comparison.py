"""The two comparison methods of Sec. 10, plain FP64 on the CPU.

Newton-Schulz, eq. (Newton-Schulz):  X_{k+1} = 2 X_k - X_k A X_k,
    started at X_0 = 0.99 A^T / rho^2(A) so that rho(I - X_0 A) < 1 (Sec. 10).
Minimal residual (MR), eq. (MRdef) / eq. (MRiter), with R_k = I - A X_k:
    X_{k+1} = X_k + alpha_k X_k R_k,
    alpha_k = Tr(R_k^T A X_k R_k) / Tr((A X_k R_k)^T A X_k R_k),
    started at the projected identity X_0 = (Tr A / Tr(A A^T)) I (Sec. 10).

rho(A): the paper takes it from MATLAB's normest (a power method for ||A||_2).  Here,
for the SPD matrices of the experiments, rho(A) = ||A||_2 is estimated by `power_norm`:
K steps of the power method on A from v_0 = (1, ..., 1)/sqrt(n), w = A v, sigma = ||w||,
v = w / sigma; the GPU runs the same K steps from the same vector, so both sides start
from the same X_0 up to rounding.  (0.99 leaves room for the estimate's shortfall.)

The stopping rule of Sec. 10 is ||I - A X_k||_F / ||I - A X_0||_F < 1e-2.
"""
import numpy as np

POWER_STEPS = 100


def power_norm(A, steps=POWER_STEPS):
    """||A||_2 of an SPD A by `steps` power-method steps from the all-ones vector."""
    n = A.shape[0]
    v = np.ones(n) / np.sqrt(n)
    sigma = 0.0
    for _ in range(steps):
        w = A @ v
        sigma = float(np.linalg.norm(w))
        v = w / sigma
    return sigma


def ns_x0(A, steps=POWER_STEPS):
    """X_0 = 0.99 A^T / rho^2(A) (Sec. 10)."""
    r = power_norm(A, steps)
    return 0.99 * A.T / (r * r)


def ns_step(X, A):
    """eq. (Newton-Schulz)."""
    return 2.0 * X - X @ A @ X


def mr_x0(A):
    """The projected identity (Tr A / Tr(A A^T)) I (Sec. 10)."""
    return (np.trace(A) / np.trace(A @ A.T)) * np.eye(A.shape[0])


def mr_alpha(X, A):
    """The step length of eq. (MRiter)."""
    R = np.eye(A.shape[0]) - A @ X
    Q = A @ X @ R
    return float(np.trace(R.T @ Q) / np.trace(Q.T @ Q))


def mr_step(X, A):
    """eq. (MRiter): X + alpha X R with R = I - A X."""
    R = np.eye(A.shape[0]) - A @ X
    return X + mr_alpha(X, A) * (X @ R)


def run(method, A, iters, X0=None, record=None):
    """`iters` steps of 'newton_schulz' or 'mr' from the paper's X_0 (or X0)."""
    A = np.asarray(A, dtype=np.float64)
    if X0 is None:
        X = ns_x0(A) if method == "newton_schulz" else mr_x0(A)
    else:
        X = np.array(X0, dtype=np.float64)
    step = ns_step if method == "newton_schulz" else mr_step
    for k in range(iters):
        X = step(X, A)
        if record is not None:
            record(k, X)
    return X
