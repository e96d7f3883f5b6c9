"""Partition sampling with the probabilities of eq. (ihsih0), plain FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A complete discrete sampling over a partition of [n] into r = n / q consecutive blocks
C_i = {i q, ..., (i+1) q - 1} (the form Sec. 9.3 assumes "for simplicity"):

  * fixed RBFGS (W = A^-1): S = I_{:C_i} with p_i = Tr(S_i^T A S_i) / Tr(S^T A S), the
    convenient probabilities of eq. (convprob) for this W (Sec. 7.3 / Sec. 9.3);
  * AdaRBFGS (Sec. 9.3, eq. siug98sUJi): S = L_k I_{:C_i}, i.e. S~ = I_{:C_i} in the
    factored step, with p_i = Tr(S_i^T A S_i) / Tr(L_k^T A L_k), recomputed from L_k at
    every iteration -- the distribution Theorem lem:9hs9hIKKK assumes.

Stream and draw (shared by specification, not by code, with the GPU side): the words of
iteration k are Philox4x64-10 of counter (0, k, 3, 0) under key (seed, 0); word 0 gives
u = ((w >> 11) + 0.5) 2^-53 in (0, 1).  Block weights w_i = sum_{j in C_i} t_j, their
running sums c_i = w_0 + ... + w_i in FP64, and the block drawn is the first i with
c_i > u c_{r-1} (the last block if rounding leaves none).  q must divide n.
"""
import numpy as np

from . import rbfgs as _rb
from .sketch import coord_matrix, stream_block

KIND_PART = 3
_TWO_M53 = 2.0 ** -53


def blocks(n, q):
    """The partition C_0, ..., C_{r-1} of [0, n) into consecutive blocks of q."""
    if q < 1 or n % q:
        raise ValueError("partition sampling needs q to divide n")
    return [np.arange(i * q, (i + 1) * q) for i in range(n // q)]


def uniform(seed, k):
    """u in (0, 1) of iteration k."""
    w = int(stream_block(seed, k, KIND_PART, 0)[0])
    return ((w >> 11) + 0.5) * _TWO_M53


def block_weights_fixed(A, q):
    """Tr(S_i^T A S_i) for S_i = I_{:C_i}."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    return np.array([np.trace(coord_matrix(C, n).T @ A @ coord_matrix(C, n)) for C in blocks(n, q)])


def block_weights_ada(L, A, q):
    """Tr(S_i^T A S_i) for S_i = L I_{:C_i} (eq. ihsih0 with S = L_k, eq. S_9898y8)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    out = []
    for C in blocks(n, q):
        Si = L @ coord_matrix(C, n)
        out.append(np.trace(Si.T @ A @ Si))
    return np.array(out)


def probabilities(weights):
    w = np.asarray(weights, dtype=np.float64)
    return w / w.sum()


def draw(weights, u):
    """First block whose running weight sum exceeds u times the total."""
    c = np.cumsum(np.asarray(weights, dtype=np.float64))
    hit = np.nonzero(c > u * c[-1])[0]
    return int(hit[0]) if hit.size else len(c) - 1


def run_fixed(A, q, seed, iters, X0=None, record=None):
    """Fixed-sketch RBFGS (eq. qunac) with S = I_{:C_i}, i drawn by the weights of A."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    parts = blocks(n, q)
    w = block_weights_fixed(A, q)
    X = np.eye(n) if X0 is None else np.array(X0, dtype=np.float64)
    for k in range(iters):
        i = draw(w, uniform(seed, k))
        X = _rb.fixed_step(X, A, coord_matrix(parts[i], n))
        if record is not None:
            record(k, X, i)
    return X


def run_ada(A, q, seed, iters, L0=None, record=None):
    """AdaRBFGS (eq. Cholimprov) with S~ = I_{:C_i}, i drawn by the weights of L_k^T A L_k."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    parts = blocks(n, q)
    L = np.eye(n) if L0 is None else np.array(L0, dtype=np.float64)
    for k in range(iters):
        i = draw(block_weights_ada(L, A, q), uniform(seed, k))
        L = _rb.ada_step(L, A, coord_matrix(parts[i], n))
        if record is not None:
            record(k, L, i)
    return L


def estimator_fixed(X, A, C, p):
    """||(I - X A) I_{:C}||_F^2 / p_C: the blocks cover every column once, so its mean over
    the draw is ||I - X A||_F^2 for any probabilities (Horvitz-Thompson)."""
    n = A.shape[0]
    S = coord_matrix(C, n)
    return float(np.sum((S - X @ (A @ S)) ** 2)) / p


def estimator_ada(L, A, C, p):
    """||(I - L^T A L) I_{:C}||_F^2 / p_C, unbiased for ||I - L^T A L||_F^2 in the same way."""
    n = A.shape[0]
    S = coord_matrix(C, n)
    return float(np.sum((S - L.T @ (A @ (L @ S))) ** 2)) / p


# ---------------------------------------------------------------- importance (eq. discoptprob)
# Simultaneous randomized Kaczmarz (Alg. 1 with W = I, eq. badbroyadj) over the same
# partition, S = I_{:C_i}, with the probabilities that minimise the bound gamma(p) of
# eq. (98h9s8h8s): p_i proportional to ||W^1/2 A^-1 Sbar_i S_i^T A W^-1/2||_F with W = I and
# Sbar_i = S_i (the partition's S is the identity), and the iterate X_k in place of the
# unknown A^-1 (the heuristic of Sec. 7.2): p_i proportional to ||X_k I_{:C_i} I_{C_i:} A||_F,
# recomputed at every iteration (for q = 1 the paper's example ||X_k e_i|| ||e_i^T A||).

def block_weights_importance(X, A, q):
    """||X I_{:C_i} I_{C_i:} A||_F for every block (eq. discoptprob with A^-1 -> X)."""
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    out = []
    for C in blocks(n, q):
        E = coord_matrix(C, n)
        out.append(np.linalg.norm(X @ E @ E.T @ A))
    return np.array(out)


def run_kaczmarz_importance(A, q, seed, iters, X0=None, record=None):
    """Kaczmarz steps (eq. badbroyadj) with S = I_{:C_i}, i drawn by the weights of X_k."""
    from . import variants as _v
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    parts = blocks(n, q)
    X = np.eye(n) if X0 is None else np.array(X0, dtype=np.float64)
    for k in range(iters):
        i = draw(block_weights_importance(X, A, q), uniform(seed, k))
        X = _v.kaczmarz_step(X, A, coord_matrix(parts[i], n))
        if record is not None:
            record(k, X, i)
    return X


def estimator_rows(X, A, C, p):
    """||I_{C:} (I - A X)||_F^2 / p_C, unbiased for ||I - A X||_F^2 (the rows of the
    blocks cover every row once)."""
    n = A.shape[0]
    S = coord_matrix(C, n)
    return float(np.sum((S.T - S.T @ A @ X) ** 2)) / p
