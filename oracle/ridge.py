"""The ridge-regression Hessian of eq. (ridgeMatrix), plain FP64 on the CPU.

f(x) = 1/2 ||B x - b||^2 + lam/2 ||x||^2 has Hessian B^T B + lam I; the benchmark's
workload scales the data term by 1/m (scale = 1/m for an m x n data matrix B).
"""
import numpy as np


def ridge_hessian(B, scale, lam):
    """scale * B^T B + lam * I (B: m x n)."""
    B = np.asarray(B, dtype=np.float64)
    return scale * (B.T @ B) + lam * np.eye(B.shape[1])


def ridge_objective_grad(B, b, lam, x, scale=1.0):
    """Gradient of scale/2 ||B x - b||^2 + lam/2 ||x||^2."""
    B = np.asarray(B, dtype=np.float64)
    return scale * (B.T @ (B @ x - b)) + lam * x
