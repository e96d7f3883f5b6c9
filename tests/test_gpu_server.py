"""Serving extension: several inversions sharing the GPU through rbfgs_server_*.

Every job's outcome in an overlapping mix must equal the same job run alone by a direct
rbfgs_invert (the path is deterministic, so iterations, residual and X agree exactly) -- with
windows of 16 iterations launched kernel by kernel, and with windows of 15 replayed as captured
HIP graphs; admission must keep the running footprints within the budget, and a job that cannot
fit is rejected at submission.
"""
import numpy as np
import pytest

from workloads import gram_ridge, spectral_spd

pytestmark = pytest.mark.gpu

JOBS = [  # (n, q, variant, precision, sketch)
    (64, 8, "adaptive", "mixed", "gauss"),
    (100, 12, "adaptive", "mixed", "coord"),
    (300, 20, "fixed", "fp64", "gauss"),
    (520, 40, "adaptive", "fp64", "gauss"),
    (257, 32, "adaptive", "mixed", "gauss"),
    (700, 64, "fixed", "mixed", "coord"),
]
TOL = 1e-2


def _matrix(j, n):
    return gram_ridge(n, 10 + j) if j % 2 == 0 else spectral_spd(n, 20 + j, 1.0, 30.0)[0].astype(np.float32)


def _direct(lib, A, q, seed, variant, precision, sketch, max_iters, check_every=16):
    with lib.Solver(A, q, seed, sketch=sketch, variant=variant, precision=precision, check_every=check_every) as s:
        ok, iters, resid = s.invert(TOL, max_iters)
        X = s.x()
    return ok, iters, resid, X


def _drain(srv, count, timeout_polls=2000):
    out = []
    for _ in range(timeout_polls):
        out += srv.poll(64, wait_ms=50)
        if len(out) >= count:
            break
    return out


@pytest.mark.parametrize("check_every", [16, 15])
def test_server_results_match_direct_solves(lib, check_every):
    import torch
    mats = [_matrix(j, n) for j, (n, *_rest) in enumerate(JOBS)]
    X = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for (n, *_rest) in JOBS]
    with lib.Server(budget_bytes=8 << 30, workers=4) as srv:
        for j, ((n, q, variant, precision, sketch), A) in enumerate(zip(JOBS, mats)):
            srv.submit(torch.from_numpy(A).cuda(), q, 100 + j, TOL, 3000, tag=j, variant=variant,
                       precision=precision, sketch=sketch, check_every=check_every, x_out=X[j])
        res = {r["tag"]: r for r in _drain(srv, len(JOBS))}
        info = srv.stats()
    assert sorted(res) == list(range(len(JOBS)))
    assert info["peak_running"] >= 2  # jobs did overlap
    for j, ((n, q, variant, precision, sketch), A) in enumerate(zip(JOBS, mats)):
        ok, iters, resid, Xd = _direct(lib, A, q, 100 + j, variant, precision, sketch, 3000, check_every)
        r = res[j]
        assert r["status"] == (lib.OK if ok else lib.E_NOT_CONVERGED), (j, r)
        assert r["iters"] == iters, (j, r, iters)
        assert r["resid"] == resid or (np.isnan(r["resid"]) and np.isnan(resid)), (j, r, resid)
        assert torch.equal(X[j], Xd), (j, float((X[j] - Xd).abs().max()))
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_server_many_jobs_each_equal_alone(lib):
    """Sixteen jobs through six slots (more slots than streams, more jobs than slots), graph
    windows: each X equals the job run alone."""
    import torch
    specs = [(64 + 37 * j, max(1, (64 + 37 * j) // 8)) for j in range(16)]
    mats = [torch.from_numpy(gram_ridge(n, 40 + j)).cuda() for j, (n, _) in enumerate(specs)]
    X = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for n, _ in specs]
    with lib.Server(budget_bytes=8 << 30, workers=6) as srv:
        for j, ((n, q), A) in enumerate(zip(specs, mats)):
            srv.submit(A, q, 300 + j, TOL, 3000, tag=j, check_every=15, x_out=X[j])
        res = {r["tag"]: r for r in _drain(srv, len(specs))}
        info = srv.stats()
    assert sorted(res) == list(range(len(specs))) and info["peak_running"] >= 4
    for j, ((n, q), A) in enumerate(zip(specs, mats)):
        ok, iters, resid, Xd = _direct(lib, A, q, 300 + j, "adaptive", "mixed", "gauss", 3000, 15)
        assert res[j]["iters"] == iters and torch.equal(X[j], Xd), j


def test_server_budget_limits_concurrency_and_returns_x(lib):
    import torch
    n, q = 256, 16
    fp = lib.rbfgs_footprint(n, q, variant="adaptive", precision="mixed")
    A = torch.from_numpy(gram_ridge(n, 3)).cuda()
    X = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(3)]
    with lib.Server(budget_bytes=fp + fp // 2, workers=4) as srv:  # room for one job at a time
        for t in range(3):
            srv.submit(A, q, 7 + t, TOL, 2000, tag=t, x_out=X[t])
        res = _drain(srv, 3)
        info = srv.stats()
    assert len(res) == 3 and all(r["status"] == lib.OK for r in res)
    assert info["peak_running"] == 1 and info["peak_bytes"] <= fp + fp // 2
    for t in range(3):
        with lib.Solver(A, q, 7 + t, variant="adaptive", precision="mixed") as s:
            s.invert(TOL, 2000)
            ref = s.x()
        assert torch.equal(X[t], ref)


def test_server_rejects_job_beyond_budget(lib):
    import torch
    n, q = 512, 32
    fp = lib.rbfgs_footprint(n, q, variant="adaptive", precision="mixed")
    A = torch.from_numpy(gram_ridge(n, 3)).cuda()
    with lib.Server(budget_bytes=fp // 2, workers=2) as srv:
        with pytest.raises(lib.RbfgsError) as e:
            srv.submit(A, q, 1, TOL, 100, tag=0)
        assert e.value.status == lib.E_OOM
        assert srv.stats()["outstanding"] == 0


def test_server_cancel_queued_and_running(lib):
    """A queued job is cancelled at once (0 iterations); a running one stops at a window
    boundary with E_CANCELLED and its X equals that of the job run alone for the same number
    of iterations; its memory returns to the pool; an unknown tag is an error."""
    import time
    import torch
    n, q, every = 1024, 64, 15
    A = torch.from_numpy(gram_ridge(n, 5)).cuda()
    X = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with lib.Server(budget_bytes=8 << 30, workers=1) as srv:
        # tolerance far below what mixed precision reaches: the job runs until cancelled
        srv.submit(A, q, 11, 1e-12, 10 ** 7, tag=0, check_every=every, x_out=X)
        srv.submit(A, q, 12, TOL, 3000, tag=1, check_every=every)  # waits behind job 0
        srv.cancel(1)
        r1 = _drain(srv, 1)
        assert len(r1) == 1 and r1[0]["tag"] == 1 and r1[0]["status"] == lib.E_CANCELLED and r1[0]["iters"] == 0
        for _ in range(400):
            if srv.stats()["running"] == 1:
                break
            time.sleep(0.005)
        time.sleep(0.3)
        srv.cancel(0)
        r0 = _drain(srv, 1)
        info = srv.stats()
        with pytest.raises(lib.RbfgsError) as e:
            srv.cancel(0)  # nothing outstanding carries the tag any more
        assert e.value.status == lib.E_INVALID_ARG
    assert len(r0) == 1 and r0[0]["status"] == lib.E_CANCELLED, r0
    k = r0[0]["iters"]
    assert k > 0 and k % every == 0, k
    assert info["outstanding"] == 0 and info["running"] == 0 and info["active_bytes"] == 0
    with lib.Solver(A, q, 11, variant="adaptive", precision="mixed", check_every=every) as s:
        s.step(k)
        ref = s.x()
    assert torch.equal(X, ref), float((X - ref).abs().max())
