"""Writes c2_fingerprint_n4096_q64_500.npz: a fingerprint of the FP64 oracle's iterate X_500 of
fixed-sketch RBFGS (eq. qunac) on the n = 4096 workload A = M^T M / 4096 + 1e-3 I (FP32), q = 64,
seed 2016, X_0 = I, for the Gaussian and the uniform-coordinate sketch.

Five hundred dense oracle steps take minutes at this size, too long for every GPU test run, so
the test compares the GPU iterate with what is stored here:
  * X_500 P for 8 seeded N(0,1) probe columns P (E ||E P||_F^2 = 8 ||E||_F^2 for any E, so the
    probed relative error estimates the relative Frobenius error);
  * ||X_500||_F, the diagonal, and 4096 seeded off-diagonal entries (for an entrywise bound).
Only the oracle and the input generator are called.

    python tests/golden/make_c2_fingerprint.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import rbfgs as R  # noqa: E402
from workloads import gram_ridge  # noqa: E402

N, Q, STEPS, SEED = 4096, 64, 500, 2016
PROBES, ENTRIES = 8, 4096
OUT = os.path.join(HERE, "c2_fingerprint_n4096_q64_500.npz")


def probes_and_entries():
    """The probe matrix and the sampled (row, col) pairs, seeded; shared with the test."""
    rng = np.random.default_rng([SEED, 77])
    P = rng.standard_normal((N, PROBES))
    rows = rng.integers(0, N, ENTRIES)
    cols = rng.integers(0, N, ENTRIES)
    return P, rows, cols


def main():
    A = np.asarray(gram_ridge(N, SEED), np.float64)
    P, rows, cols = probes_and_entries()
    out = {}
    for kind in ("gauss", "cols"):
        X = R.run_fixed(A, Q, SEED, kind, STEPS,
                        record=lambda k, X: print(f"{kind} step {k + 1}", flush=True) if (k + 1) % 50 == 0 else None)
        out[f"{kind}_XP"] = X @ P
        out[f"{kind}_fro"] = np.array(np.linalg.norm(X))
        out[f"{kind}_diag"] = np.diag(X).copy()
        out[f"{kind}_entries"] = X[rows, cols]
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
