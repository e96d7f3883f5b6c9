"""Closed forms and brute-force references used to pin the oracle.

  * `Z_matrix`, `expected_Z`, `rho` -- eq. (Z) and eq. (rhoequiv) of Sec. 6 with
    W = A^-1 (the BFGS choice of Table tbl:QN):
        Z = A S (S^T A S)^-1 S^T A,   rho = 1 - lambda_min(A^-1/2 E[Z] A^-1/2).
    For a discrete distribution E[Z] is the probability-weighted sum over the
    outcomes (Prop. 7.1, eq. EZdiscrete).
  * `rho_single_coordinate` -- the same rho for S = e_i with p_i = 1/n:
    E[Z] = (1/n) sum_i A e_i e_i^T A / A_ii, hence
    rho = 1 - lambda_min(D^-1/2 A D^-1/2) / n with D = diag(A).
  * `projection_kkt` -- eq. (NFsym) solved as a dense equality-constrained
    least-squares problem over the n(n+1)/2 free entries of a symmetric X,
    with no use of the closed form (tiny n only).
"""
import itertools

import numpy as np


def _sym_inv_sqrt(A):
    w, Q = np.linalg.eigh(A)
    return Q @ np.diag(w ** -0.5) @ Q.T


def Z_matrix(A, S):
    """Z = A S (S^T A W A S)^-1 S^T A with W = A^-1 (eq. Z)."""
    AS = A @ S
    return AS @ np.linalg.solve(S.T @ AS, AS.T)


def expected_Z(A, outcomes, probs):
    """E[Z] for a discrete sketch distribution: sum_i p_i Z(S_i)."""
    EZ = np.zeros_like(A, dtype=np.float64)
    for S, p in zip(outcomes, probs):
        EZ += p * Z_matrix(A, S)
    return EZ


def rho_from_EZ(A, EZ):
    """rho = 1 - lambda_min(W^1/2 E[Z] W^1/2) with W = A^-1 (eq. rhoequiv)."""
    Wh = _sym_inv_sqrt(A)
    M = Wh @ EZ @ Wh
    return 1.0 - float(np.linalg.eigvalsh(0.5 * (M + M.T))[0])


def uniform_subsets(n, q):
    """All q-subsets of [0, n) as coordinate sketches, each with probability 1/C(n,q)."""
    subsets = list(itertools.combinations(range(n), q))
    outs = []
    for c in subsets:
        S = np.zeros((n, q))
        S[list(c), range(q)] = 1.0
        outs.append(S)
    return outs, [1.0 / len(subsets)] * len(subsets)


def rho_single_coordinate(A):
    """Closed form of rho for S = e_i drawn uniformly (derived from eq. EZdiscrete)."""
    n = A.shape[0]
    d = 1.0 / np.sqrt(np.diag(A))
    M = d[:, None] * A * d[None, :]
    return 1.0 - float(np.linalg.eigvalsh(M)[0]) / n


def projection_kkt(Xk, A, S):
    """argmin_X 1/2 ||X - Xk||_{F(A)}^2  s.t.  S^T A X = S^T,  X = X^T  (eq. NFsym, W = A^-1).

    X is parametrised by its lower triangle theta (vec(X) = D theta).  The
    objective is 1/2 (D theta - x_k)^T (A kron A) (D theta - x_k), the
    constraint (I kron S^T A) D theta = vec(S^T) (column-major vec).  The KKT
    system is solved by least squares because symmetric X makes q(q-1)/2 of the
    constraints redundant.
    """
    n, q = S.shape
    pairs = [(i, j) for j in range(n) for i in range(j, n)]
    D = np.zeros((n * n, len(pairs)))
    for t, (i, j) in enumerate(pairs):
        D[i + j * n, t] = 1.0
        D[j + i * n, t] = 1.0
    H = np.kron(A, A)
    C = np.kron(np.eye(n), S.T @ A) @ D
    b = S.T.reshape(-1, order="F")
    xk = Xk.reshape(-1, order="F")
    m = len(pairs)
    K = np.zeros((m + C.shape[0], m + C.shape[0]))
    K[:m, :m] = D.T @ H @ D
    K[:m, m:] = C.T
    K[m:, :m] = C
    rhs = np.concatenate([D.T @ H @ xk, b])
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    return (D @ sol[:m]).reshape(n, n, order="F")


def projection_kkt_weighted(Xk, A, S, Winv, symmetric):
    """argmin_X 1/2 ||X - Xk||_{F(W^-1)}^2  s.t.  S^T A X = S^T  (and X = X^T when
    `symmetric`): eq. (NF) (row variant) or eq. (NFsym), for a general weight.

    ||X||_{F(W^-1)}^2 = Tr(X^T W^-1 X W^-1) = vec(X)^T (W^-1 kron W^-1) vec(X)
    (column-major vec, W symmetric).  X is parametrised by all n^2 entries, or by
    its lower triangle when symmetric; the KKT system is solved by least squares
    (some constraints are redundant under the symmetry constraint).
    """
    n, q = S.shape
    if symmetric:
        pairs = [(i, j) for j in range(n) for i in range(j, n)]
        D = np.zeros((n * n, len(pairs)))
        for t, (i, j) in enumerate(pairs):
            D[i + j * n, t] = 1.0
            D[j + i * n, t] = 1.0
    else:
        D = np.eye(n * n)
    H = np.kron(Winv, Winv)
    C = np.kron(np.eye(n), S.T @ A) @ D
    b = S.T.reshape(-1, order="F")
    xk = Xk.reshape(-1, order="F")
    m = D.shape[1]
    K = np.zeros((m + C.shape[0], m + C.shape[0]))
    K[:m, :m] = D.T @ H @ D
    K[:m, m:] = C.T
    K[m:, :m] = C
    rhs = np.concatenate([D.T @ H @ xk, b])
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    return (D @ sol[:m]).reshape(n, n, order="F")
