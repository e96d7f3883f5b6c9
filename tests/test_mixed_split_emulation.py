"""CPU emulation of the mixed-precision fixed-sketch step (Sec. 8.7, eq. qunac) against the FP64
oracle: the arithmetic the bf16 kernels apply, written out in numpy -- FP32 operands presented as
bf16 pieces (round to nearest even, each piece the rounding of what the previous ones leave), the
piece products of total weight >= 2^-(8 pmax) kept, FP32 sums -- with the q-sized products in FP64
as the library computes them for q > n/8.  It pins the choice of pieces for the symmetric update
X+ = X - (U W'^T + W' U^T): with q/n = 1/4 on the ridge Hessian (kappa ~ 1e6), U and W' in two
pieces leave the iterate above the 1e-4 mixed bar and three pieces bring it below, while at
q/n = 1/8 two pieces suffice; the library takes three pieces exactly when q > n/8.

Test infrastructure only: nothing here runs or imports the HIP path.
"""
import numpy as np
import pytest

from oracle import rbfgs as R, sketch as sk
from workloads import ridge_hessian


def bf16(x):
    """Round FP32 values to bf16 (nearest, ties to even), returned as FP32."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def pieces(x, n):
    out, rest = [], np.asarray(x, np.float32)
    for _ in range(n):
        h = bf16(rest)
        out.append(h)
        rest = (rest - h).astype(np.float32)
    return out


def split_product(Ap, Bp, pmax):
    """sum over piece pairs with pa + pb <= pmax of Ap[pa] @ Bp[pb], smallest weights first, FP32."""
    acc = np.zeros((Ap[0].shape[0], Bp[0].shape[1]), np.float32)
    for lvl in range(pmax, -1, -1):
        for pa in range(len(Ap)):
            pb = lvl - pa
            if 0 <= pb < len(Bp):
                acc = (acc + (Ap[pa] @ Bp[pb]).astype(np.float32)).astype(np.float32)
    return acc


def mixed_step(X, A32, S, upd_pieces):
    """One step: Y = A S (exact bf16 S, FP32 sums), G, U = S G^-1, V = X Y (2 x 2 pieces),
    H = Y^T V and W' = V - S/2 - U H/2 in FP64 (q > n/8), and the symmetric update with U and W'
    in upd_pieces pieces each (pmax = pieces - 1), X kept in FP32."""
    Y = (A32 @ S).astype(np.float32)
    G = S.T.astype(np.float64) @ Y.astype(np.float64)
    U = (S @ np.linalg.inv(G).astype(np.float32)).astype(np.float32)
    V = split_product(pieces(X, 2), pieces(Y, 2), 1)
    H = Y.astype(np.float64).T @ V.astype(np.float64)
    W = (V - S / 2 - (U.astype(np.float64) @ H) / 2).astype(np.float32)
    P, Q = np.concatenate([U, W], 1), np.concatenate([W, U], 1)
    D = split_product(pieces(P, upd_pieces), [p.T.copy() for p in pieces(Q, upd_pieces)], upd_pieces - 1)
    return (X - D).astype(np.float32)


def run_emulated(A, q, seed, steps, upd_pieces):
    n = A.shape[0]
    A32 = np.asarray(A, np.float32)
    X = np.eye(n, dtype=np.float32)
    for k in range(steps):
        X = mixed_step(X, A32, sk.sketch(seed, k, n, q, "gauss").astype(np.float32), upd_pieces)
    return X


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_three_bf16_pieces_represent_fp32_exactly():
    """hi + mid + lo of an FP32 value (normal range) is the value: 3 x 8 significant bits."""
    x = (np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-6, 6, 10000))
    x = x.astype(np.float32)
    h, m, l = pieces(x, 3)
    assert np.array_equal((h.astype(np.float64) + m + l).astype(np.float32), x)
    h2, l2 = pieces(x, 2)
    assert np.max(np.abs((h2.astype(np.float64) + l2 - x) / x)) <= 2.0 ** -16


@pytest.mark.slow
def test_update_pieces_rule_at_large_q_over_n():
    """n = 1024, q = 256 (q/n = 1/4), 40 steps: two pieces > 1e-4 > three pieces; n = 2048, q = 256
    (q/n = 1/8): two pieces < 1e-4."""
    A = ridge_hessian(1024, 5, m=2048, lam=1e-2)
    Xo = R.run_fixed(np.asarray(A, np.float64), 256, 2, "gauss", 40)
    e2 = rel(run_emulated(A, 256, 2, 40, 2), Xo)
    e3 = rel(run_emulated(A, 256, 2, 40, 3), Xo)
    assert e2 > 1e-4 > e3, (e2, e3)
    A8 = ridge_hessian(2048, 5, m=4096, lam=1e-2)
    Xo8 = R.run_fixed(np.asarray(A8, np.float64), 256, 2, "gauss", 40)
    assert rel(run_emulated(A8, 256, 2, 40, 2), Xo8) < 1e-4
