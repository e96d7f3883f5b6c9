"""Pins of the FP64 oracle against the paper's mathematics (CPU only).

Each test checks the oracle against something other than itself: a library
routine, a closed form, an invariant stated by the paper, a brute-force solve,
or an exact enumeration of a discrete distribution.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.stats
import torch

from oracle import philox, rbfgs as R, sketch as sk, theory as T
from workloads import (spectral_spd, gram_ridge, householder_spd, householder_entries,
                       ridge_hessian)


def spd(n, seed=0, lo=1.0, hi=50.0):
    return spectral_spd(n, seed, lo, hi)


# ------------------------------------------------------------------ RNG pins
@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((5, 7, 0, 0), (1, 2)),
                                     ((2 ** 64 - 1, 3, 9, 11), (2 ** 63 + 5, 77)),
                                     ((12345, 2 ** 40, 1, 0), (987654321, 0))])
def test_philox_matches_numpy(ctr, key):
    """Philox4x64-10 block == numpy.random.Philox.random_raw (which increments first)."""
    ref = np.random.Philox(counter=np.array(ctr, dtype=np.uint64),
                           key=np.array(key, dtype=np.uint64)).random_raw(8)
    c0 = (ctr[0] + 1) % 2 ** 64
    c1 = ctr[1] + (1 if ctr[0] == 2 ** 64 - 1 else 0)
    out = philox.philox4x64(np.uint64(c0), np.uint64(c1), np.uint64(ctr[2]), np.uint64(ctr[3]),
                            np.uint64(key[0]), np.uint64(key[1]))
    assert [int(v) for v in out] == [int(v) for v in ref[:4]]
    c0b = (ctr[0] + 2) % 2 ** 64
    c1b = ctr[1] + (1 if ctr[0] >= 2 ** 64 - 2 else 0)
    out2 = philox.philox4x64(np.uint64(c0b), np.uint64(c1b), np.uint64(ctr[2]), np.uint64(ctr[3]),
                             np.uint64(key[0]), np.uint64(key[1]))
    assert [int(v) for v in out2] == [int(v) for v in ref[4:]]


def test_mulhilo_against_python_ints():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 2 ** 63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    hi, lo = philox.mulhilo64(a, b)
    for x, y, h, l in zip(a[:200], b[:200], hi[:200], lo[:200]):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


def test_bf16_rounding_matches_torch():
    """Values exact in FP32 round like torch's FP32 -> bfloat16 (RNE) conversion."""
    rng = np.random.default_rng(1)
    x32 = (rng.standard_normal(200000) * np.exp(rng.uniform(-5, 5, 200000))).astype(np.float32)
    # force many exact ties: 8 significant bits + half ulp
    ties = (np.round(rng.standard_normal(5000) * 128) + 0.5).astype(np.float32) / np.float32(64)
    x32 = np.concatenate([x32, ties, -ties])
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = sk.round_bf16(x32.astype(np.float64))
    np.testing.assert_array_equal(got, ref)


def test_gaussian_sketch_distribution():
    S = sk.gaussian_sketch(11, 3, 4096, 16)
    z = S.reshape(-1)
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1) < 0.02
    # bf16 rounding moves the CDF by < 2^-9 relative; KS at this size is insensitive to it
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # every entry is a bf16 value (8 significant bits)
    np.testing.assert_array_equal(sk.round_bf16(z), z)
    # independence across iterations and seeds
    S2 = sk.gaussian_sketch(11, 4, 4096, 16)
    S3 = sk.gaussian_sketch(12, 3, 4096, 16)
    assert abs(np.corrcoef(z, S2.reshape(-1))[0, 1]) < 0.02
    assert abs(np.corrcoef(z, S3.reshape(-1))[0, 1]) < 0.02


def test_gaussian_sketch_layout():
    """Entry e = j*n + i of the column-major sketch comes from block e>>2, word e&3."""
    n, q, seed, k = 37, 5, 99, 7
    S = sk.gaussian_sketch(seed, k, n, q)
    for (i, j) in [(0, 0), (1, 0), (36, 0), (0, 1), (13, 4), (36, 4)]:
        e = j * n + i
        w = [int(v) for v in sk.stream_block(seed, k, sk.KIND_GAUSS, e >> 2)]
        p = (e & 3) >> 1
        ua = ((w[2 * p] >> 11) + 0.5) * 2.0 ** -53
        ub = ((w[2 * p + 1] >> 11) + 0.5) * 2.0 ** -53
        r = math.sqrt(-2.0 * math.log(ua))
        z = r * (math.cos(2 * math.pi * ub) if (e & 1) == 0 else math.sin(2 * math.pi * ub))
        assert S[i, j] == float(sk.round_bf16(np.array([z]))[0])


def test_lemire_bounded_uniform():
    st = sk._WordStream(5, 0, sk.KIND_COLS)
    m = 7
    counts = np.bincount([sk.bounded(st, m) for _ in range(70000)], minlength=m)
    assert scipy.stats.chisquare(counts).pvalue > 1e-4
    # m = 2^63 + 1 has rejection probability ~ 1/2: result stays in range
    big = 2 ** 63 + 1
    assert all(0 <= sk.bounded(st, big) < big for _ in range(200))


def test_coord_sketch_uniform_over_subsets():
    """Floyd sampling gives every q-subset with equal probability (exhaustive for n=6, q=2)."""
    n, q = 6, 2
    counts = {c: 0 for c in itertools.combinations(range(n), q)}
    for k in range(15000):
        idx = sk.coord_sketch(3, k, n, q)
        assert len(set(idx)) == q and list(idx) == sorted(idx)
        counts[tuple(int(v) for v in idx)] += 1
    assert scipy.stats.chisquare(list(counts.values())).pvalue > 1e-4


@pytest.mark.parametrize("n,q", [(1, 1), (5, 5), (100, 1), (1000, 64), (16384, 256)])
def test_coord_sketch_edges(n, q):
    idx = sk.coord_sketch(17, 2, n, q)
    assert len(idx) == q and len(set(idx.tolist())) == q
    assert idx.min() >= 0 and idx.max() < n and np.all(np.diff(idx) > 0)
    if q == n:
        np.testing.assert_array_equal(idx, np.arange(n))


# ---------------------------------------------------------- fixed-step pins
@pytest.mark.parametrize("kind", ["gauss", "cols"])
def test_factored_equals_literal(kind):
    """P1: the thin-factor evaluation equals eq. (qunac) as printed."""
    A, _ = spd(48, 1)
    X = np.eye(48)
    for k in range(5):
        S = sk.sketch(7, k, 48, 6, kind)
        Xa = R.fixed_step(X, A, S)
        Xb = R.fixed_step_literal(X, A, S)
        assert np.linalg.norm(Xa - Xb) <= 1e-12 * np.linalg.norm(Xb)
        X = Xb


@pytest.mark.parametrize("n,q", [(3, 1), (5, 2), (6, 3)])
def test_brute_force_projection(n, q):
    """P16: eq. (NFsym) solved by a dense KKT system equals the closed-form step."""
    A, _ = spd(n, n + q)
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    X = M @ M.T + np.eye(n)
    S = sk.gaussian_sketch(4, 0, n, q)
    Xkkt = T.projection_kkt(X, A, S)
    Xf = R.fixed_step(X, A, S)
    assert np.abs(Xkkt - Xf).max() <= 1e-9 * np.abs(Xf).max()


@pytest.mark.parametrize("kind", ["gauss", "cols"])
def test_invariants_along_trajectory(kind):
    """P2 sketched equation, P3 symmetry/SPD, P4 Pythagoras, P8 error recursion."""
    n, q = 40, 5
    A, Ainv = spd(n, 2)
    X = np.eye(n)
    for k in range(30):
        S = sk.sketch(21, k, n, q, kind)
        Xn = R.fixed_step(X, A, S)
        # P2: X_{k+1} A S = S
        assert np.linalg.norm(Xn @ A @ S - S) <= 1e-11 * np.linalg.norm(S)
        # P3
        assert np.array_equal(Xn, Xn.T)
        np.linalg.cholesky(Xn)
        # P4: projection onto an affine set containing A^-1, in the F(A) norm
        e0, e1, d = R.error_FA(X, A, Ainv), R.error_FA(Xn, A, Ainv), R.error_FA(Xn, A, X)
        assert abs(e0 ** 2 - (e1 ** 2 + d ** 2)) <= 1e-10 * e0 ** 2
        assert e1 <= e0 * (1 + 1e-12)
        # P8: X_{k+1} - A^-1 = (I - W Z)(X_k - A^-1)(I - Z W), W = A^-1
        Z = T.Z_matrix(A, S)
        I = np.eye(n)
        rhs = (I - Ainv @ Z) @ (X - Ainv) @ (I - Z @ Ainv)
        assert np.linalg.norm(Xn - Ainv - rhs) <= 1e-9 * np.linalg.norm(X - Ainv)
        X = Xn


def test_idempotent_and_fixed_point():
    """P5 re-applying the same S changes nothing; P6 A^-1 is a fixed point."""
    A, Ainv = spd(30, 3)
    S = sk.gaussian_sketch(1, 0, 30, 4)
    X1 = R.fixed_step(np.eye(30), A, S)
    assert np.abs(R.fixed_step(X1, A, S) - X1).max() <= 1e-11 * np.abs(X1).max()
    assert np.abs(R.fixed_step(Ainv, A, S) - Ainv).max() <= 1e-11 * np.abs(Ainv).max()


@pytest.mark.parametrize("kind", ["gauss", "cols"])
def test_one_step_when_q_equals_n(kind):
    """P7 (Sec. 8.1): an invertible S gives X_1 = A^-1 from any start."""
    n = 12
    A, Ainv = spd(n, 4)
    S = sk.sketch(9, 0, n, n, kind)
    X1 = R.fixed_step(5 * np.eye(n), A, S)
    assert np.abs(X1 - Ainv).max() <= 1e-10 * np.abs(Ainv).max()


def test_not_spd_detected():
    with pytest.raises(R.NotSPDError):
        R.fixed_step(np.eye(4), -np.eye(4), sk.gaussian_sketch(0, 0, 4, 2))


# ------------------------------------------------------------------ rate pins
def test_rho_bounds_and_closed_form():
    """eq. (rholower) 1 - q/n <= rho <= 1; q = 1 uniform coordinates closed form."""
    n = 6
    A, _ = spd(n, 5)
    rho1 = T.rho_from_EZ(A, T.expected_Z(A, *T.uniform_subsets(n, 1)))
    assert abs(rho1 - T.rho_single_coordinate(A)) < 1e-12
    for q in (1, 2, 3):
        rho = T.rho_from_EZ(A, T.expected_Z(A, *T.uniform_subsets(n, q)))
        assert 1 - q / n - 1e-12 <= rho <= 1 + 1e-12


@pytest.mark.parametrize("q", [1, 2])
def test_expected_error_contracts_by_rho_exact(q):
    """Thm 6.2 (Enormconv) for the symmetric method, checked by exact enumeration.

    E ||X_1 - A^-1||_{F(A)}^2 over all equally likely q-subsets <= rho ||X_0 - A^-1||^2,
    and the same over all pairs of subsets for two steps (<= rho^2).
    """
    n = 6
    A, Ainv = spd(n, 6, 1.0, 20.0)
    outs, probs = T.uniform_subsets(n, q)
    rho = T.rho_from_EZ(A, T.expected_Z(A, outs, probs))
    X0 = np.eye(n)
    e0 = R.error_FA(X0, A, Ainv) ** 2
    e1 = sum(p * R.error_FA(R.fixed_step(X0, A, S), A, Ainv) ** 2 for S, p in zip(outs, probs))
    assert e1 <= rho * e0 * (1 + 1e-12)
    e2 = 0.0
    for S1, p1 in zip(outs, probs):
        X1 = R.fixed_step(X0, A, S1)
        for S2, p2 in zip(outs, probs):
            e2 += p1 * p2 * R.error_FA(R.fixed_step(X1, A, S2), A, Ainv) ** 2
    assert e2 <= rho ** 2 * e0 * (1 + 1e-12)


@pytest.mark.slow
def test_linear_rate_monte_carlo_with_sampler():
    """Thm 6.2 with the oracle's own coordinate sampler (q = 1), averaged over seeds."""
    n, q, K, seeds = 8, 1, 12, 400
    A, Ainv = spd(n, 7, 1.0, 10.0)
    rho = T.rho_single_coordinate(A)
    e0 = R.error_FA(np.eye(n), A, Ainv) ** 2
    errs = np.zeros(K)
    for s in range(seeds):
        def rec(k, X):
            errs[k] += R.error_FA(X, A, Ainv) ** 2 / seeds
        R.run_fixed(A, q, s, "cols", K, record=rec)
    bound = e0 * rho ** np.arange(1, K + 1)
    assert np.all(errs <= bound * 1.10)


# ----------------------------------------------------------------- estimator
def test_estimator_unbiased_exact_for_coordinates():
    """P14: averaging the estimator over all q-subsets gives ||I - XA||_F^2 exactly."""
    n = 6
    A, _ = spd(n, 8)
    X = np.diag(np.linspace(0.1, 1.0, n))
    truth = np.linalg.norm(np.eye(n) - X @ A) ** 2
    for q in (1, 2, 3):
        outs, probs = T.uniform_subsets(n, q)
        avg = sum(p * R.estimator(X, A, S, "cols") for S, p in zip(outs, probs))
        assert abs(avg - truth) <= 1e-12 * truth


def test_estimator_unbiased_gaussian():
    n, q = 50, 4
    A, _ = spd(n, 9)
    X = 0.01 * np.eye(n)
    truth = np.linalg.norm(np.eye(n) - A @ X) ** 2
    ests = [R.estimator(X, A, sk.gaussian_sketch(s, 0, n, q), "gauss") for s in range(400)]
    assert abs(np.mean(ests) - truth) <= 0.05 * truth


# ------------------------------------------------------------------ AdaRBFGS
@pytest.mark.parametrize("kind", ["gauss", "cols"])
def test_ada_factor_is_rbfgs_step(kind):
    """P10: L+ L+^T equals one RBFGS step on X = L L^T with S = L S~, for both
    square-root choices; the algorithm box's literal R_k = (S~^T A S~)^-1/2 does not."""
    n, q = 20, 4
    A, _ = spd(n, 10)
    rng = np.random.default_rng(3)
    L = np.linalg.cholesky(np.eye(n) + 0.1 * (lambda M: M @ M.T)(rng.standard_normal((n, n))))
    St = sk.sketch(2, 0, n, q, kind)
    Xref = R.fixed_step(L @ L.T, A, L @ St)
    for step in (R.ada_step, R.ada_step_sqrt):
        Ln = step(L, A, St)
        assert np.abs(Ln @ Ln.T - Xref).max() <= 1e-11 * np.abs(Xref).max()
    # literal reading of the algorithm box
    S = L @ St
    w, Q = np.linalg.eigh(St.T @ A @ St)
    Rlit = Q @ np.diag(w ** -0.5) @ Q.T
    w2, Q2 = np.linalg.eigh(St.T @ St)
    C = Q2 @ np.diag(w2 ** -0.5) @ Q2.T
    Llit = L + S @ Rlit @ (C @ St.T - Rlit.T @ S.T @ A @ L)
    assert np.abs(Llit @ Llit.T - Xref).max() > 1e-3 * np.abs(Xref).max()


def test_ada_cyclic_partition_terminates():
    """P11: with S~ running through a partition of [n], L^T A L = I after n/q steps."""
    n, q = 24, 4
    A, Ainv = spd(n, 11)
    L = np.eye(n)
    for b in range(n // q):
        L = R.ada_step(L, A, sk.coord_matrix(np.arange(b * q, (b + 1) * q), n))
    assert np.abs(L.T @ A @ L - np.eye(n)).max() <= 1e-9
    assert np.abs(L @ L.T - Ainv).max() <= 1e-9 * np.abs(Ainv).max()


def test_ada_estimator_exact_for_coordinates():
    n = 6
    A, _ = spd(n, 12)
    L = np.diag(np.linspace(0.5, 1.5, n))
    truth = np.linalg.norm(np.eye(n) - L.T @ A @ L) ** 2
    outs, probs = T.uniform_subsets(n, 2)
    avg = sum(p * R.ada_estimator(L, A, S, "cols") for S, p in zip(outs, probs))
    assert abs(avg - truth) <= 1e-12 * truth


@pytest.mark.parametrize("kind", ["gauss", "cols"])
def test_ada_converges_and_keeps_spd(kind):
    n, q = 64, 8
    A, Ainv = spd(n, 13, 1.0, 1e3)
    r0 = R.residual_fro(A, np.eye(n))
    L = R.run_ada(A, q, 5, kind, 120)
    X = L @ L.T
    np.linalg.cholesky(X)
    assert R.residual_fro(A, X) < 1e-3 * r0


# ----------------------------------------------------------------- workloads
def test_closed_form_inverses():
    """P13: the generators' exact inverses match a library inverse."""
    A, Ainv = spectral_spd(64, 1)
    np.testing.assert_allclose(Ainv, np.linalg.inv(A), rtol=0, atol=1e-12 * np.abs(Ainv).max())
    Ah = householder_spd(200, 2, r=16, dtype=np.float64)
    Ahi = householder_spd(200, 2, r=16, dtype=np.float64, inverse=True)
    np.testing.assert_allclose(Ahi, np.linalg.inv(Ah), rtol=0, atol=1e-10 * np.abs(Ahi).max())
    rows, cols = np.array([0, 5, 199, 17]), np.array([0, 9, 3, 17])
    np.testing.assert_allclose(householder_entries(200, 2, rows, cols, r=16, inverse=True),
                               Ahi[rows, cols], rtol=1e-12, atol=1e-14)
    Ar = ridge_hessian(64, 3, m=128)
    assert Ar.dtype == np.float32 and np.array_equal(Ar, Ar.T)
    np.linalg.cholesky(Ar.astype(np.float64))
    Ag = gram_ridge(64, 4)
    assert np.array_equal(Ag, Ag.T)


def test_fixed_rbfgs_converges_to_closed_form_inverse():
    n, q = 64, 8
    A, Ainv = spectral_spd(n, 2, 1.0, 30.0)
    e0 = np.linalg.norm(np.eye(n) - Ainv)
    X = R.run_fixed(A, q, 1, "gauss", 150)
    assert np.linalg.norm(X - Ainv) < 1e-2 * e0


def test_first_step_entries_match_dense_step():
    """The entry formula for X_1 from X_0 = I equals the dense step of eq. (qunac)."""
    from oracle import rbfgs as R, sketch as sk
    n, q = 40, 7
    A, _ = spectral_spd(n, 3, 1.0, 50.0)
    S = sk.gaussian_sketch(5, 0, n, q)
    X1 = R.fixed_step_literal(np.eye(n), A, S)
    rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    got = R.first_step_entries(A.astype(np.float32), S, rows.ravel(), cols.ravel(), block=16)
    ref = R.fixed_step_literal(np.eye(n), A.astype(np.float32).astype(np.float64), S)
    assert np.abs(got - ref.ravel()).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(R.first_step_entries(A, S, rows.ravel(), cols.ravel()) - X1.ravel()).max() <= 1e-12 * np.abs(X1).max()


def test_householder_large_n_exactly_symmetric():
    """The row-block construction used above n = 8192 stores an exactly symmetric matrix
    (the library checks symmetry on the stored values)."""
    A = householder_spd(8448, 3, r=8, row_block=2048)
    assert np.array_equal(A, A.T)
