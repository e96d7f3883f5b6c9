"""Preconditioned conjugate gradients for A x = b with an approximate inverse as the
preconditioner -- the use of X ~ A^-1 the paper motivates (Sec. 1) -- plain FP64 on the CPU.

The textbook method (Hestenes & Stiefel 1952; Saad, Iterative Methods for Sparse Linear
Systems, Alg. 9.1), started at x_0 = 0 with preconditioner application z = M r
(M = I gives plain CG):
    r_0 = b, z_0 = M r_0, p_0 = z_0
    alpha_k = (r_k . z_k) / (p_k . A p_k);  x_{k+1} = x_k + alpha_k p_k;  r_{k+1} = r_k - alpha_k A p_k
    z_{k+1} = M r_{k+1};  beta_k = (r_{k+1} . z_{k+1}) / (r_k . z_k);  p_{k+1} = z_{k+1} + beta_k p_k
"""
import numpy as np


def pcg(A, b, M=None, iters=None, tol=None, max_iters=100000, record=None):
    """Run `iters` iterations, or until ||r_k|| <= tol ||b|| (checked every iteration).
    Returns (x, k, ||r_k|| / ||b||)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    apply_m = (lambda r: r) if M is None else (lambda r: M @ r)
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_m(r)
    p = z.copy()
    rz = float(r @ z)
    nb = float(np.linalg.norm(b))
    limit = iters if iters is not None else max_iters
    k = 0
    while k < limit:
        if tol is not None and np.linalg.norm(r) <= tol * nb:
            break
        Ap = A @ p
        alpha = rz / float(p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = apply_m(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        k += 1
        if record is not None:
            record(k, x, r)
    return x, k, float(np.linalg.norm(r)) / nb
