"""GPU parity of partition sampling with the probabilities of eq. (ihsih0) through the C ABI
against the FP64 oracle: the draw itself (bit-exact block indices), fixed RBFGS and
AdaRBFGS iterates (1e-10 FP64, 1e-4 mixed), the device-kept AdaRBFGS weights
diag(L^T A L), their recomputation after rbfgs_set_state, and the estimator."""
import math

import numpy as np
import pytest

from oracle import partition as Pt
from workloads import gram_ridge, spectral_spd

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,q", [(4096, 64), (4096, 1), (300, 3), (96, 96), (1 << 14, 256)])
def test_draw_matches_oracle(lib, n, q):
    import torch
    rng = np.random.default_rng(n + q)
    t = rng.random(n) ** 3
    if n // q > 4:
        t[q: 3 * q] = 0.0  # zero-weight blocks are never drawn
    w = t.reshape(n // q, q).sum(1)
    td = torch.from_numpy(t).cuda()
    for k in range(60):
        idx, ht = lib.rbfgs_sample_partition(td, q, 11, k)
        i = Pt.draw(w, Pt.uniform(11, k))
        got = idx.cpu().numpy()
        assert np.array_equal(got, np.arange(i * q, (i + 1) * q)), (k, got[0] // q, i)
        assert abs(float(ht.cpu()[0]) - w.sum() / w[i]) <= 1e-12 * w.sum() / w[i]


def test_draw_rejects_ragged(lib):
    import torch
    with pytest.raises(lib.RbfgsError):
        lib.rbfgs_sample_partition(torch.ones(10, dtype=torch.float64, device="cuda"), 4, 1, 0)


@pytest.mark.parametrize("n,q,steps", [(256, 16, 40), (513, 27, 30), (300, 300, 1), (64, 1, 50)])
def test_fixed_fp64_parity(lib, n, q, steps):
    A, _ = spectral_spd(n, n + q, 1.0, 100.0)
    with lib.Solver(A, q, 3, sketch="partition") as s:
        s.step(steps)
        X = s.x().cpu().numpy()
        t = s.weights()
    assert rel(X, Pt.run_fixed(A, q, 3, steps)) <= FP64_TOL
    assert np.array_equal(t, np.diag(A))


@pytest.mark.parametrize("n,q,steps", [(256, 16, 20), (513, 27, 12), (64, 1, 40)])
def test_ada_fp64_parity(lib, n, q, steps):
    A, _ = spectral_spd(n, 2 * n + q, 1.0, 100.0)
    with lib.Solver(A, q, 5, sketch="partition", variant="adaptive") as s:
        s.step(steps)
        L = s.factor().cpu().numpy()
        t = s.weights()
    Lo = Pt.run_ada(A, q, 5, steps)
    assert rel(L, Lo) <= FP64_TOL
    d = np.diag(Lo.T @ A @ Lo)
    assert np.abs(t - d).max() <= FP64_TOL * np.abs(d).max()


@pytest.mark.parametrize("variant", ["fixed", "adaptive"])
def test_mixed_parity(lib, variant):
    n, q = 520, 40
    A = gram_ridge(n, 6)
    steps = 60 if variant == "fixed" else 30
    with lib.Solver(A, q, 2, sketch="partition", variant=variant, precision="mixed") as s:
        s.step(steps)
        X = s.x().cpu().numpy()
        t = s.weights()
        if variant == "adaptive":
            Lg = s.factor().cpu().numpy()
    A64 = np.asarray(A, np.float64)
    if variant == "fixed":
        Xo = Pt.run_fixed(A64, q, 2, steps)
        assert np.array_equal(t, np.diag(A64))
    else:
        Lo = Pt.run_ada(A64, q, 2, steps)
        Xo = Lo @ Lo.T
        d = np.diag(Lg.T @ A64 @ Lg)  # the weights the device keeps for its own L
        assert np.abs(t - d).max() <= MIXED_TOL * np.abs(d).max()
    assert rel(X, Xo) <= MIXED_TOL


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_set_state_recomputes_ada_weights(lib, precision, tol):
    """After rbfgs_set_state the weights are diag(L^T A L) of the new L (n^3 recomputation),
    and resuming reproduces the uninterrupted run."""
    n, q = 256, 32
    A = gram_ridge(n, 3)
    with lib.Solver(A, q, 4, sketch="partition", variant="adaptive", precision=precision) as s:
        s.step(6)
        L6 = s.factor().cpu().numpy()
        t6 = s.weights()
        s.step(4)
        L10 = s.factor().cpu().numpy()
    with lib.Solver(A, q, 4, sketch="partition", variant="adaptive", precision=precision) as r:
        r.set_state(L6, 6)
        t = r.weights()
        r.step(4)
        L10r = r.factor().cpu().numpy()
    assert np.abs(t - t6).max() <= tol * np.abs(t6).max()
    assert rel(L10r, L10) <= tol


@pytest.mark.parametrize("variant", ["fixed", "adaptive"])
def test_estimator_matches_oracle(lib, variant):
    """The estimate of the last step: ||(I - M) I_{:C}||_F^2 / p_C for the iterate it
    started from and the block it drew (Horvitz-Thompson)."""
    n, q, steps = 200, 20, 7
    A, _ = spectral_spd(n, 12, 1.0, 50.0)
    rec = {}
    if variant == "fixed":
        Pt.run_fixed(A, q, 8, steps - 1, record=lambda k, X, i: rec.update(X=X))
        X = rec["X"]
        w = Pt.block_weights_fixed(A, q)
        i = Pt.draw(w, Pt.uniform(8, steps - 1))
        ref = Pt.estimator_fixed(X, A, Pt.blocks(n, q)[i], w[i] / w.sum())
    else:
        Pt.run_ada(A, q, 8, steps - 1, record=lambda k, L, i: rec.update(L=L))
        L = rec["L"]
        w = Pt.block_weights_ada(L, A, q)
        i = Pt.draw(w, Pt.uniform(8, steps - 1))
        ref = Pt.estimator_ada(L, A, Pt.blocks(n, q)[i], w[i] / w.sum())
    with lib.Solver(A, q, 8, sketch="partition", variant=variant) as s:
        s.step(steps)
        est = s.estimate()
    assert abs(est - ref) <= 1e-9 * ref


@pytest.mark.parametrize("variant", ["fixed", "adaptive"])
def test_invert_converges(lib, variant):
    n, q = 96, 12
    A, _ = spectral_spd(n, 6, 1.0, 30.0)
    with lib.Solver(A, q, 1, sketch="partition", variant=variant, check_every=4) as s:
        ok, iters, resid = s.invert(tol=1e-8, max_iters=20000)
        assert ok and resid <= 1e-8
        X = s.x().cpu().numpy()
    assert np.linalg.norm(np.eye(n) - A @ X) / math.sqrt(n) <= 1e-8


def test_rejected_uses(lib):
    A, _ = spectral_spd(64, 1)
    for variant in ("psb", "aip", "kaczmarz", "newton_schulz"):
        with pytest.raises(lib.RbfgsError) as ei:
            lib.Solver(A, 8, 1, sketch="partition", variant=variant)
        assert ei.value.status == lib.E_INVALID_ARG
    with pytest.raises(lib.RbfgsError):
        lib.Solver(A, 6, 1, sketch="partition")  # 6 does not divide 64
    with lib.Solver(A, 8, 1) as s:
        with pytest.raises(lib.RbfgsError):
            s.weights()


# ---------------------------------------------------------------- importance (eq. discoptprob)
def general_matrix(n, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / math.sqrt(n) + 2.5 * np.eye(n)
    return np.ascontiguousarray(A.astype(dtype))


@pytest.mark.parametrize("n,q,steps", [(96, 12, 30), (256, 32, 20), (64, 1, 40)])
def test_importance_fp64_parity(lib, n, q, steps):
    A = general_matrix(n, n + q)
    rec = {}
    Xo = Pt.run_kaczmarz_importance(A, q, 7, steps, record=lambda k, X, i: rec.update({k: X}))
    with lib.Solver(A, q, 7, sketch="importance", variant="kaczmarz") as s:
        s.step(steps)
        X = s.x().cpu().numpy()
        t = s.weights()
    assert rel(X, Xo) <= FP64_TOL
    Xprev = rec[steps - 2] if steps > 1 else np.eye(n)  # the last draw used X_{steps-1}
    w = Pt.block_weights_importance(Xprev, A, q)
    assert np.abs(t[::q] - w).max() <= FP64_TOL * w.max()
    assert not np.any(t.reshape(-1, q)[:, 1:])


@pytest.mark.parametrize("n,q,precision", [(1200, 100, "fp64"), (1088, 64, "mixed"), (1000, 20, "fp64"),
                                           (1200, 200, "fp64"), (600, 300, "mixed"), (1024, 256, "mixed")])
def test_importance_weights_span_tiles(lib, n, q, precision):
    """The block weights at sizes whose Grams span several tiles (q = 100, 200, 256, 300), several
    chunks of the n-long sums with a ragged last chunk, and the narrow-tile form (q = 20):
    weights of a seeded non-symmetric X_k set by rbfgs_set_state against the oracle's
    ||X_k I_{:C_i} I_{C_i:} A||_F on the same (stored-precision) X_k and A."""
    dt = np.float64 if precision == "fp64" else np.float32
    A = general_matrix(n, n + q, dt)
    X0 = np.eye(n) + np.random.default_rng(n).standard_normal((n, n)) / (4 * math.sqrt(n))
    X0 = X0.astype(dt).astype(np.float64)
    with lib.Solver(A, q, 3, sketch="importance", variant="kaczmarz", precision=precision) as s:
        s.set_state(X0, 5)
        s.step(1)
        t = s.weights()
    w = Pt.block_weights_importance(X0, np.asarray(A, np.float64), q)
    assert np.abs(t[::q] - w).max() <= FP64_TOL * w.max()
    assert not np.any(t.reshape(-1, q)[:, 1:])


def test_importance_mixed_parity(lib):
    n, q, steps = 520, 40, 30
    A = general_matrix(n, 3, np.float32)
    with lib.Solver(A, q, 2, sketch="importance", variant="kaczmarz", precision="mixed") as s:
        s.step(steps)
        X = s.x().cpu().numpy()
    Xo = Pt.run_kaczmarz_importance(np.asarray(A, np.float64), q, 2, steps)
    assert rel(X, Xo) <= MIXED_TOL


def test_importance_estimator_matches_oracle(lib):
    n, q, steps = 120, 12, 6
    A = general_matrix(n, 5)
    rec = {}
    Pt.run_kaczmarz_importance(A, q, 9, steps - 1, record=lambda k, X, i: rec.update(X=X))
    X = rec["X"]
    w = Pt.block_weights_importance(X, A, q)
    i = Pt.draw(w, Pt.uniform(9, steps - 1))
    ref = Pt.estimator_rows(X, A, Pt.blocks(n, q)[i], w[i] / w.sum())
    with lib.Solver(A, q, 9, sketch="importance", variant="kaczmarz") as s:
        s.step(steps)
        est = s.estimate()
    assert abs(est - ref) <= 1e-9 * ref


def test_importance_invert_and_resume(lib):
    n, q = 96, 12
    A = general_matrix(n, 6)
    with lib.Solver(A, q, 1, sketch="importance", variant="kaczmarz", check_every=4) as s:
        ok, iters, resid = s.invert(tol=1e-8, max_iters=20000)
        assert ok and resid <= 1e-8
    with lib.Solver(A, q, 1, sketch="importance", variant="kaczmarz") as s:
        s.step(5)
        X5 = s.x().cpu().numpy()
        s.step(5)
        X10 = s.x().cpu().numpy()
    with lib.Solver(A, q, 1, sketch="importance", variant="kaczmarz") as r:
        r.set_state(X5, 5)
        r.step(5)
        assert rel(r.x().cpu().numpy(), X10) <= FP64_TOL


def test_importance_rejected_uses(lib):
    A = general_matrix(64, 1)
    As, _ = spectral_spd(64, 1)
    for variant in ("fixed", "adaptive", "psb", "aip"):
        with pytest.raises(lib.RbfgsError):
            lib.Solver(As, 8, 1, sketch="importance", variant=variant)
    with pytest.raises(lib.RbfgsError):
        lib.Solver(A, 6, 1, sketch="importance", variant="kaczmarz")
