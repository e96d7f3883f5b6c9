"""GPU parity of CG preconditioned with the context's approximate inverse, through the C ABI,
against the FP64 oracle PCG run with the same preconditioner."""
import numpy as np
import pytest

from oracle import pcg as P
from workloads import gram_ridge, spectral_spd

pytestmark = pytest.mark.gpu

NEVER = 1e-300  # a tolerance no run reaches: exactly max_iters iterations


def rhs(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def rounding_bar(A, b, M, iters):
    """CG amplifies rounding differences along its trajectory (more so with a poor
    preconditioner early in the iteration, where kappa(X A) can exceed kappa(A)).  The
    bar is ten times the oracle's own relative movement when b is perturbed by sqrt(n) u,
    the size of one reordered dot product's rounding, floored at 1e-10."""
    n = b.shape[0]
    x0, _, _ = P.pcg(A, b, M=M, iters=iters)
    pert = 1.1e-16 * np.sqrt(n) * np.random.default_rng(0).standard_normal(n)
    x1, _, _ = P.pcg(A, b * (1.0 + pert), M=M, iters=iters)
    return max(1e-10, 10.0 * np.linalg.norm(x1 - x0) / np.linalg.norm(x0))


@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("n,steps,iters", [(1, 1, 1), (37, 3, 10), (300, 5, 25), (513, 4, 40)])
def test_fixed_fp64_parity(lib, precond, n, steps, iters):
    A, _ = spectral_spd(n, n, 1.0, 1e3)
    b = rhs(n, n)
    with lib.Solver(A, max(1, n // 8), 2) as s:
        s.step(steps)
        X = s.x().cpu().numpy()
        x, ok, k, rel = s.pcg(b, precond=precond, tol=NEVER, max_iters=iters)
    xo, ko, relo = P.pcg(A, b, M=X if precond else None, iters=iters)
    assert k == iters and ko == iters
    bar = rounding_bar(A, b, X if precond else None, iters)
    assert bar <= 1e-6  # the case still measures parity
    dx = np.linalg.norm(x.cpu().numpy() - xo)
    assert dx <= bar * np.linalg.norm(xo)
    # r = b - A x away from the rounding floor: | ||r|| - ||r_o|| | <= ||A||_2 ||x - x_o||
    assert abs(rel - relo) * np.linalg.norm(b) <= 1.01 * np.linalg.norm(A, 2) * dx + 1e-14


def test_adaptive_factor_preconditioner_parity(lib):
    """AdaRBFGS applies M = L L^T as L (L^T r)."""
    n = 400
    A, _ = spectral_spd(n, 3, 1.0, 1e3)
    b = rhs(n, 3)
    with lib.Solver(A, 40, 5, variant="adaptive") as s:
        s.step(8)
        L = s.factor().cpu().numpy()
        x, ok, k, rel = s.pcg(b, tol=NEVER, max_iters=30)
    xo, _, _ = P.pcg(A, b, M=L @ L.T, iters=30)
    bar = rounding_bar(A, b, L @ L.T, 30)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= bar * np.linalg.norm(xo)


def test_mixed_context_parity(lib):
    """Mixed mode stores A and X in FP32; the products run in FP64 on those values."""
    n = 520
    A = gram_ridge(n, 6)
    b = rhs(n, 6)
    with lib.Solver(A, 40, 1, precision="mixed") as s:
        s.step(10)
        X = s.x().cpu().numpy()
        x, ok, k, rel = s.pcg(b, tol=NEVER, max_iters=20)
    A64 = np.asarray(A, np.float64)
    xo, _, _ = P.pcg(A64, b, M=X, iters=20)
    bar = rounding_bar(A64, b, X, 20)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= bar * np.linalg.norm(xo)


def test_preconditioner_pays_off(lib):
    """After enough iterations X is a good approximate inverse: PCG needs far fewer
    iterations than CG on an ill-conditioned A."""
    n = 256
    A, Ainv = spectral_spd(n, 9, 1.0, 1e4)
    b = rhs(n, 9)
    with lib.Solver(A, 64, 3, variant="adaptive") as s:
        ok, it, resid = s.invert(tol=1e-2, max_iters=5000)
        assert ok
        _, ok0, k0, _ = s.pcg(b, precond=False, tol=1e-8, max_iters=5000)
        x, ok1, k1, rel = s.pcg(b, precond=True, tol=1e-8, max_iters=5000)
    assert ok0 and ok1 and k1 * 3 <= k0
    assert np.linalg.norm(x.cpu().numpy() - Ainv @ b) <= 1e-6 * np.linalg.norm(Ainv @ b)


def test_invalid_uses_rejected(lib):
    A, _ = spectral_spd(32, 1)
    for variant in ("psb", "kaczmarz"):
        with lib.Solver(A, 4, 1, variant=variant) as s:
            with pytest.raises(lib.RbfgsError) as ei:
                s.pcg(rhs(32, 1))
            assert ei.value.status == lib.E_INVALID_ARG
    with lib.Solver(A, 4, 1, variant="aip") as s:  # an SPD A: plain CG is fine, X as M is not
        _, ok, _, _ = s.pcg(rhs(32, 1), precond=False)
        assert ok
        with pytest.raises(lib.RbfgsError):
            s.pcg(rhs(32, 1), precond=True)


@pytest.mark.parametrize("variant", ["fixed", "adaptive"])
def test_mixed_end_to_end_against_oracle_preconditioner(lib, variant):
    """End to end in mixed precision: the GPU's own iterate (30 mixed steps) preconditions the
    GPU's CG, the oracle's own FP64 iterate (30 oracle steps on the same FP32 A) preconditions
    the oracle's CG; both run to ||r|| <= 1e-8 ||b||.  The two preconditioners differ at the
    mixed-precision level (about 1e-5), so the iteration counts agree up to the GPU's test
    interval (every 8 iterations), and both solutions lie within kappa(A) * tol of A^-1 b."""
    from oracle import rbfgs as R
    n, q, steps, tol = 520, 40, 30, 1e-8
    A = gram_ridge(n, 9)
    A64 = np.asarray(A, np.float64)
    b = rhs(n, 9)
    with lib.Solver(A, q, 4, variant=variant, precision="mixed") as s:
        s.step(steps)
        x, ok, k, rel = s.pcg(b, precond=True, tol=tol, max_iters=2000)
    if variant == "fixed":
        Mo = R.run_fixed(A64, q, 4, "gauss", steps)
    else:
        Lo = R.run_ada(A64, q, 4, "gauss", steps)
        Mo = Lo @ Lo.T
    xo, ko, relo = P.pcg(A64, b, M=Mo, tol=tol, max_iters=2000)
    assert ok and relo <= tol
    assert ko <= k <= (ko + 7) // 8 * 8 + 8, (k, ko)
    xs = np.linalg.solve(A64, b)
    w = np.linalg.eigvalsh(A64)
    bound = 2.0 * (w[-1] / w[0]) * tol * np.linalg.norm(xs)
    x = x.cpu().numpy()
    assert np.linalg.norm(x - xs) <= bound and np.linalg.norm(xo - xs) <= bound
    assert np.linalg.norm(b - A64 @ x) <= 1.01 * tol * np.linalg.norm(b)
