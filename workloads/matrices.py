"""Generators for the synthetic workloads (see package docstring)."""
import math

import numpy as np


def _rng(seed, tag):
    return np.random.default_rng([int(seed), int(tag)])


def spectral_spd(n, seed, lam_min=1.0, lam_max=1e3):
    """A = Q diag(lambda) Q^T (FP64) and its exact inverse.

    Q from numpy's QR of a seeded N(0,1) n x n matrix; lambda_i log-uniform in
    [lam_min, lam_max].  Returns (A, A_inv), both symmetrised.
    """
    rng = _rng(seed, 1)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.exp(rng.uniform(math.log(lam_min), math.log(lam_max), n))
    A = (Q * lam) @ Q.T
    Ainv = (Q / lam) @ Q.T
    return 0.5 * (A + A.T), 0.5 * (Ainv + Ainv.T)


def gram_ridge(n, seed, mu=1e-3, dtype=np.float32, device=None):
    """A = M^T M / n + mu I with M a seeded N(0,1) n x n matrix, rounded to `dtype`.

    M is drawn on the host; the FP64 Gram product runs on `device` (a torch device
    string) when given, with the same result up to the rounding order."""
    rng = _rng(seed, 2)
    M = rng.standard_normal((n, n), dtype=np.float64)
    if device is not None:
        import torch
        Mt = torch.from_numpy(M).to(device)
        A = (Mt.T @ Mt) / n
        A.diagonal().add_(mu)
        A = 0.5 * (A + A.T)
        out = A.to(torch.float32 if dtype == np.float32 else torch.float64).cpu().numpy()
        del Mt, A
        return out
    A = (M.T @ M) / n
    A[np.diag_indices(n)] += mu
    A = 0.5 * (A + A.T)
    return A.astype(dtype)


def ridge_data(n, seed, m=None, scale_lo=1e-2, scale_hi=1e2):
    """The m x n FP32 data matrix B = N(0,1) times diag(d), d log-uniform in
    [scale_lo, scale_hi] (heterogeneous feature scales), of the ridge workload."""
    if m is None:
        m = 2 * n
    rng = _rng(seed, 3)
    d = np.exp(rng.uniform(math.log(scale_lo), math.log(scale_hi), n))
    B = rng.standard_normal((m, n), dtype=np.float32)
    B *= d.astype(np.float32)[None, :]
    return B


def ridge_hessian(n, seed, m=None, lam=1e-2, scale_lo=1e-2, scale_hi=1e2,
                  dtype=np.float32, device=None):
    """A = B^T B / m + lam I with B from `ridge_data`.

    B is drawn on the host (seeded numpy stream, FP32 normal draws promoted to
    FP64).  The Gram product is formed in FP64, on `device` (a torch device
    string) when given -- for n = 16384, m = 32768 it is a 1.8e13-flop product --
    otherwise with numpy.  The result is symmetrised and rounded to `dtype`.
    """
    if m is None:
        m = 2 * n
    B = ridge_data(n, seed, m, scale_lo, scale_hi)
    if device is not None:
        import torch
        Bt = torch.from_numpy(B).to(device=device, dtype=torch.float64)
        A = (Bt.T @ Bt) / m
        A.diagonal().add_(lam)
        A = 0.5 * (A + A.T)
        out = A.to(torch.float32 if dtype == np.float32 else torch.float64).cpu().numpy()
        del Bt, A
        return out
    B64 = B.astype(np.float64)
    A = (B64.T @ B64) / m
    A[np.diag_indices(n)] += lam
    A = 0.5 * (A + A.T)
    return A.astype(dtype)


def householder_factors(n, seed, r=64, lam_lo=1e-2, lam_hi=1e2):
    """(lam, V, T) with Q = H_1 H_2 ... H_r = I - V T V^T.

    H_j = I - tau_j v_j v_j^T, v_j ~ N(0, I), tau_j = 2 / v_j^T v_j.  T is the
    upper-triangular compact-WY factor accumulated one reflector at a time:
    (I - V T V^T)(I - tau v v^T) = I - [V v] [[T, -tau T V^T v], [0, tau]] [V v]^T.
    """
    rng = _rng(seed, 4)
    lam = np.exp(rng.uniform(math.log(lam_lo), math.log(lam_hi), n))
    V = rng.standard_normal((n, r))
    T = np.zeros((r, r))
    for j in range(r):
        v = V[:, j]
        tau = 2.0 / float(v @ v)
        if j:
            T[:j, j] = -tau * (T[:j, :j] @ (V[:, :j].T @ v))
        T[j, j] = tau
    return lam, V, T


def _wy_lowrank(lam, V, T):
    """(Ubar, C) with Q diag(lam) Q^T = diag(lam) + Ubar C Ubar^T, Q = I - V T V^T."""
    W = lam[:, None] * V                     # diag(lam) V
    M = V.T @ W                              # V^T diag(lam) V
    r = V.shape[1]
    C = np.zeros((2 * r, 2 * r))
    C[:r, :r] = T @ M @ T.T
    C[:r, r:] = -T
    C[r:, :r] = -T.T
    return np.hstack([V, W]), C


def householder_spd(n, seed, r=64, lam_lo=1e-2, lam_hi=1e2, dtype=np.float32,
                    inverse=False, row_block=4096):
    """A = Q diag(lambda) Q^T (or its exact inverse) with Q a product of r reflectors.

    Built in row blocks as diag + Ubar C Ubar^T so the FP64 intermediate never
    exceeds one block; returned as `dtype`.
    """
    lam, V, T = householder_factors(n, seed, r, lam_lo, lam_hi)
    if inverse:
        lam = 1.0 / lam
    Ub, C = _wy_lowrank(lam, V, T)
    UC = Ub @ C
    out = np.empty((n, n), dtype=dtype)
    for r0 in range(0, n, row_block):
        r1 = min(n, r0 + row_block)
        blk = UC[r0:r1] @ Ub.T
        blk[np.arange(r1 - r0), np.arange(r0, r1)] += lam[r0:r1]
        out[r0:r1] = blk.astype(dtype)
    # exact symmetry of the stored matrix (the FP64 blocks are symmetric to rounding)
    if n <= 8192:
        out = np.tril(out) + np.tril(out, -1).T
    else:
        for r0 in range(0, n, row_block):
            r1 = min(n, r0 + row_block)
            d = out[r0:r1, r0:r1]
            out[r0:r1, r0:r1] = np.tril(d) + np.tril(d, -1).T
            out[r0:r1, r1:] = out[r1:, r0:r1].T
    return out


def householder_entries(n, seed, rows, cols, r=64, lam_lo=1e-2, lam_hi=1e2, inverse=False):
    """Selected FP64 entries of the exact A (or A^-1) of `householder_spd`."""
    lam, V, T = householder_factors(n, seed, r, lam_lo, lam_hi)
    if inverse:
        lam = 1.0 / lam
    Ub, C = _wy_lowrank(lam, V, T)
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    vals = np.einsum("ij,jk,ik->i", Ub[rows], C, Ub[cols])
    vals = vals + np.where(rows == cols, lam[rows], 0.0)
    return vals


def serving_trace(njobs, seed, rate, n_lo=64, n_hi=8192, mu=1e-3):
    """Poisson arrivals (rate jobs/s) of jobs with n log-uniform in [n_lo, n_hi].

    Returns a list of dicts {id, t_arrive, n, q, seed}; q = min(256, n // 8);
    each job's matrix is gram_ridge(n, seed).
    """
    rng = _rng(seed, 5)
    gaps = rng.exponential(1.0 / rate, njobs)
    t = np.cumsum(gaps) - gaps[0]
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), njobs))).astype(int)
    seeds = rng.integers(1, 2 ** 31, njobs)
    return [dict(id=j, t_arrive=float(t[j]), n=int(ns[j]), q=int(min(256, ns[j] // 8)),
                 seed=int(seeds[j])) for j in range(njobs)]


CONFIGS = {
    "c1_n256_fp64": dict(n=256, q=16, iters=300, family="spectral", lam=(1.0, 1e3)),
    "c2_n4096": dict(n=4096, q=64, iters=500, family="gram_ridge"),
    "c3_n16384_ridge": dict(n=16384, m=32768, q=256, family="ridge_hessian", tol=1e-3),
    "c4_n32768_householder": dict(n=32768, q=(32, 512), iters=200, family="householder"),
    "c5_serving": dict(njobs=512, n=(64, 8192), family="gram_ridge", tol=1e-3,
                       budget_bytes=200 * 2 ** 30),
}
