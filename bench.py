#!/usr/bin/env python
"""Benchmark of the RBFGS hot path on one MI355X.

Workload: the ill-conditioned ridge Hessian A = B^T B / m + lam I (n = 16384,
m = 32768, columns of the Gaussian B scaled log-uniformly in [1e-2, 1e2],
lam = 1e-2), FP32 A resident in HBM, sketch size q = 256.  A step is one full
RBFGS iteration (sketch, A S, G and its Cholesky-based inverse, X A S, the q x q
products, the estimator and the symmetric rank-2q update of X).

Prints ONE JSON line: iterations/s of the mixed-precision path (value), the FP64
GPU path beside it, effective TFLOP/s from the algorithmic flop count, the
roofline figure of the dominant kernel timed live with HIP events on the
library's stream, and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--variant fixed|adaptive] [--sketch gauss|coord]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    """Progress line on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def alg_flops(n, q, variant, sketch):
    """Algorithmic flops of one iteration (products counted once, symmetric update on one triangle).

    fixed/gauss: A S, X Y (2 n^2 q each), rank-2q update on n(n+1)/2 entries (2 n^2 q),
                 G, H, S G^-1, U H (2 n q^2 each)
    fixed/coord: X Y (2 n^2 q) and the row/column update (4 n q), H, G^-1 H, R = G^-1 W'^T
    adaptive/gauss: L S~, A S, L^T Y, rank-q update of L (2 n^2 q each) + 4 panel products (2 n q^2)
    adaptive/coord: A S, L^T Y, update (2 n^2 q each) + 2 panel products
    psb: as fixed/gauss plus S^T Y (2 n q^2); coordinates applied as dense 0/1 matrices
    aip, kaczmarz: P = A S (or A^T S), X^T P, rank-q update of all of X (2 n^2 q each),
                   G and U (2 n q^2 each)
    """
    n2q, nq2 = 2.0 * n * n * q, 2.0 * n * q * q
    if variant == "psb":
        return 3 * n2q + 5 * nq2
    if variant in ("aip", "kaczmarz"):
        return 3 * n2q + 2 * nq2
    if variant == "fixed":
        return 3 * n2q + 4 * nq2 if sketch == "gauss" else n2q + 2 * nq2 + 4.0 * n * q
    return 4 * n2q + 4 * nq2 if sketch == "gauss" else 3 * n2q + 2 * nq2


def phase_roofline(name, n, q, variant, sketch, precision="mixed"):
    """(bound, algorithmic bytes per launch, unit) of one n x n product kernel.

    Bytes count each operand once at its stored width (4 B in mixed mode, 8 B in FP64):
      AS, XY, LS, LtY, XtP (tall-skinny, M(n x n) * P(n x q)): read M once, read P,
                       write the n x q result                       -> e n^2 + 2 e n q
      update (fixed, PSB): read and write the lower triangle of X (the method's own bytes:
                       the mixed fixed path keeps X on its lower tiles), read the two
                       n x 2q bf16 hi/lo panel pairs                -> e n^2 + 16 n q
      update (adaptive, AIP, Kaczmarz): read and write L (or X), read the panels
                                                                    -> 2 e n^2 + 8 n q
    Their intensity (2 n^2 q algorithmic flops over these bytes) is below the bf16
    ridge point (2500 TFLOP/s / 8 TB/s = 312 flop/B) for q <= 256, so the roofline
    that bounds them is HBM bandwidth.
    """
    e = 4.0 if precision == "mixed" else 8.0
    nn, nq = float(n) * n, float(n) * q
    if name in ("AS", "XY", "LS", "LtY", "XtP"):
        return "hbm", e * nn + 2 * e * nq, "GB/s"
    if name == "update":
        if variant in ("fixed", "psb"):
            return "hbm", e * nn + 16 * nq, "GB/s"
        return "hbm", 2 * e * nn + 8 * nq, "GB/s"
    return None


# kernel symbol (as rocprofv3 names it) of each product phase in mixed mode at n = 16384,
# q = 256: fixed RBFGS with the Gaussian sketch, and AdaRBFGS ("ada." phases)
PHASE_KERNEL = {
    "XY": "k_tall_stream<256, 2, 2, 1, 2>",
    "AS": "k_tall_stream<256, 3, 1, 2, 0>",
    "update": "k_symupd_dma<256, 32, 2, 1, 2, 4, false, 1, false, 2>",
    "ada.LS": "k_tall_stream<256, 3, 1, 2, 0>",
    "ada.AS": "k_tall_stream<256, 3, 2, 2, 0>",
    "ada.LtY": "k_tall_stream<256, 2, 3, 2, 1>",
    "ada.update": "k_symupd_dma<128, 32, 2, 2, 2, 2, true, 1, true, 2>",
}
KERNEL_SOURCES = ["paper_1602_01768_amd/csrc/k_bf16.hip", "paper_1602_01768_amd/csrc/k_tall.hip",
                  "paper_1602_01768_amd/csrc/k_symupd.hip", "paper_1602_01768_amd/csrc/common.hpp",
                  "paper_1602_01768_amd/csrc/kernels.hpp"]
COUNTERS_FILE = "profiles/hbm_counters_c3_n16384_q256_mixed.txt"


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(phase):
    """HBM bytes per launch of the phase's kernel from the committed rocprofv3 counter
    summary: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) each scaled by the factor the
    same counter reads for a copy kernel of known size.  Rows are keyed by phase (the fixed
    method's, or "ada." and the adaptive method's).  None when the summary is missing, does
    not cover the phase, or was taken from different kernel sources."""
    path = os.path.join(ROOT, COUNTERS_FILE)
    if phase not in PHASE_KERNEL or not os.path.exists(path):
        return None
    kv, rows = {}, {}
    for line in open(path):
        line = line.strip()
        if line.startswith("sources_sha256=") or line.startswith("fetch_factor=") or line.startswith("write_factor="):
            k, v = line.split("=", 1)
            kv[k] = v
        elif line.startswith("kernel="):
            f = dict(x.split("=", 1) for x in line.split(" | "))
            rows[f["phase"]] = f
    if kv.get("sources_sha256") != sources_sha256() or phase not in rows:
        return None
    r = rows[phase]
    return (float(r["fetch_kib"]) * float(kv["fetch_factor"]) + float(r["write_kib"]) * float(kv["write_factor"])) * 1024.0


def make_A(n, seed, torch, rbfgs, cpu_n=4096):
    """The C3 ridge Hessian A = B^T B / m + 1e-2 I (m = 2n), formed by the library's
    ridge-Hessian step (eq. ridgeMatrix, FP64 MFMA) from the seeded FP32 data matrix.
    Returns A on the device (FP32), on the host, and the step's timing, its FP64-MFMA
    roofline, a sampled check of 64 entries against FP64 dot products of B's columns,
    and the oracle timed on an n = cpu_n, m = 2 cpu_n sample."""
    import numpy as np
    from oracle import ridge
    from workloads import ridge_data
    m = 2 * n
    t0 = time.perf_counter()
    B = ridge_data(n, seed, m=m)
    t_data = time.perf_counter() - t0
    Bd = torch.from_numpy(B).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A_dev = rbfgs.rbfgs_ridge_hessian(Bd, 1.0 / m, 1e-2, dtype=rbfgs.F32)
    torch.cuda.synchronize()
    t_form = time.perf_counter() - t0
    del Bd
    A32 = A_dev.cpu().numpy()
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, n, size=(64, 2))
    idx[:8, 1] = idx[:8, 0]  # some diagonal entries
    err = 0.0
    for i, j in idx:
        ref = float(B[:, i].astype(np.float64) @ B[:, j].astype(np.float64)) / m + (1e-2 if i == j else 0.0)
        err = max(err, abs(float(A32[i, j]) - ref) / abs(ref))
    flops = float(n) * (n + 1) * m  # lower triangle with the diagonal, 2 flops per multiply-add
    Bs = B[: 2 * min(cpu_n, n), : min(cpu_n, n)]
    t0 = time.perf_counter()
    ridge.ridge_hessian(Bs, 1.0 / Bs.shape[0], 1e-2)
    t_cpu = time.perf_counter() - t0
    fl_cpu = float(Bs.shape[1]) ** 2 * Bs.shape[0] * 2
    info = {"seconds": round(t_form, 4), "data_gen_s": round(t_data, 2),
            "tflops": round(flops / t_form / 1e12, 2),
            "roofline": {"bound": "mfma", "achieved": round(flops / t_form / 1e12, 2), "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(flops / t_form / 1e12 / FP64_PEAK_TFLOPS, 4),
                         "traffic": None, "alg_flops": flops},
            "sampled_parity_max_rel_err": err,
            "cpu_oracle": {"value": round(fl_cpu / t_cpu / 1e12, 4), "unit": "TFLOP/s", "seconds": round(t_cpu, 3),
                           "sample": f"numpy FP64 B^T B/m + lam I at n={Bs.shape[1]}, m={Bs.shape[0]}"}}
    return A_dev, A32, info


def reference_A(n, seed, torch):
    """The same ridge Hessian formed without the library (torch's FP64 GEMM on the host-drawn
    B), for the oracle leg: the oracle's input does not come from the path it checks."""
    from workloads import ridge_data
    m = 2 * n
    B = torch.from_numpy(ridge_data(n, seed, m=m)).cuda().to(torch.float64)
    A = B.T @ B
    del B
    A /= m
    A.diagonal().add_(1e-2)
    A32 = A.to(torch.float32)
    del A
    torch.cuda.synchronize()
    return A32


def timed_steps(Solver, A_dev, q, seed, sketch, variant, precision, warmup, steps, torch, events=False):
    """Warm up, then time `steps` iterations.  With events, the n x n product kernels are
    bracketed by HIP events on the stream each runs on during the timed steps."""
    s = Solver(A_dev, q, seed, sketch=sketch, variant=variant, precision=precision)
    s.step(warmup)
    s.sync()
    if events:
        s.profile(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = s.profile_report() if events else {}
    if events:
        s.profile(0)
    return s, (t1 - t0), rep


def serving(args, torch, rbfgs):
    """C5: a trace of independent inversions to ||I - AX||_F / sqrt(n) <= tol through the
    server (AdaRBFGS, Gaussian sketch, mixed precision; A_j = M^T M / n + 1e-3 I with n_j
    log-uniform in [64, 8192], q_j = min(256, n_j / 8)).

    1. closed loop: every job submitted at t = 0; saturation throughput = jobs / makespan;
    2. open loop: Poisson arrivals at 0.7 x the saturation rate; sojourn = done - arrival,
       service = done - admission into a slot;
    3. baseline: the same arrivals served one at a time in FP64.
    The matrices are formed and resident in HBM before any timing.
    """
    import numpy as np
    from workloads import serving_trace, gram_ridge
    unit = serving_trace(args.serve_jobs, args.seed, rate=1.0)
    mats = {j["id"]: torch.from_numpy(gram_ridge(j["n"], j["seed"], device="cuda")).cuda() for j in unit}
    torch.cuda.synchronize()
    budget = int(args.serve_budget_gb * 2 ** 30)

    def run(arrivals, precision, workers):
        res = []
        with rbfgs.Server(budget, workers) as srv:
            start = time.perf_counter()
            for j, ta in zip(unit, arrivals):
                while True:
                    wait = ta - (time.perf_counter() - start)
                    if wait <= 0:
                        break
                    res += srv.poll(256, wait_ms=max(1, int(min(wait, 0.05) * 1000)))
                srv.submit(mats[j["id"]], j["q"], j["seed"], args.serve_tol, 20000, tag=j["id"],
                           variant="adaptive", precision=precision, sketch="gauss", check_every=15)
            reported = 0
            while len(res) < len(unit):
                res += srv.poll(256, wait_ms=50)
                if len(res) >= reported + 64 or len(res) == len(unit):
                    reported = len(res)
                    log(f"serving {precision} ({workers} slots): {len(res)}/{len(unit)} jobs done, "
                        f"{time.perf_counter() - start:.1f} s")
            makespan = time.perf_counter() - start
            peak = srv.stats()["peak_running"]
        return res, makespan, peak

    def summary(res, makespan, peak):
        soj = np.array([r["t_done"] - r["t_submit"] for r in res])
        svc = np.array([r["t_done"] - r["t_admit"] for r in res])
        its = sum(r["iters"] for r in res)
        conv = sum(1 for r in res if r["status"] == rbfgs.OK)
        worst = max((r["resid"] for r in res if r["status"] == rbfgs.OK), default=float("nan"))
        return {"jobs": len(res), "converged": conv, "max_resid": float(worst), "makespan_s": round(makespan, 3),
                "jobs_per_s": round(len(res) / makespan, 2), "iters_per_s": round(its / makespan, 1),
                "sojourn_p50_ms": round(1e3 * float(np.percentile(soj, 50)), 2),
                "sojourn_p99_ms": round(1e3 * float(np.percentile(soj, 99)), 2),
                "service_p50_ms": round(1e3 * float(np.percentile(svc, 50)), 2),
                "service_p99_ms": round(1e3 * float(np.percentile(svc, 99)), 2), "peak_running": peak}

    closed = run([0.0] * len(unit), "mixed", args.serve_workers)
    sat = len(unit) / closed[1]
    rate = 0.7 * sat
    arrivals = [j["t_arrive"] / rate for j in unit]
    open_mixed = run(arrivals, "mixed", args.serve_workers)
    base = run(arrivals, "fp64", 1) if args.serve_baseline else None
    out = {"workload": f"{len(unit)} AdaRBFGS jobs (gauss), n log-uniform in [64, 8192], q = min(256, n/8), "
                       f"tol {args.serve_tol}, device pool = budget {args.serve_budget_gb} GiB, "
                       f"{args.serve_workers} slots on {min(args.serve_workers, 4)} streams, windows of 15 "
                       f"iterations replayed as HIP graphs",
           "saturation_jobs_per_s": round(sat, 2), "arrival_rate_jobs_per_s": round(rate, 2),
           "closed_loop": summary(*closed), "mixed": summary(*open_mixed),
           "fp64_one_at_a_time": summary(*base) if base else None}
    del mats
    return out


def pcg_section(s, A_dev, A32, seed, torch, tol=1e-8, cap=20000, cpu_n=4096, cpu_iters=40):
    """A x = b by CG and by CG preconditioned with the AdaRBFGS iterate X = L L^T of the
    open context s: iterations, wall time, the true residual ||b - A x|| / ||b|| (FP64),
    and each iteration's HBM roofline -- the algorithmic bytes are the matrices it reads
    (A; with the preconditioner also L and L^T: 3 n^2 entries), the FP64 vectors ignored.
    The oracle's PCG is timed beside it on the leading cpu_n x cpu_n block of A."""
    import numpy as np
    from oracle import pcg as P
    n = A_dev.shape[0]
    b = torch.from_numpy(np.random.default_rng(seed + 7).standard_normal(n)).cuda()
    A64 = A_dev.to(torch.float64)
    out = {"tol": tol}
    for name, pre in (("cg", False), ("pcg_X", True)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, ok, k, rel = s.pcg(b, precond=pre, tol=tol, max_iters=cap)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        true_rel = float(torch.linalg.vector_norm(b - A64 @ x) / torch.linalg.vector_norm(b))
        per_it = t / max(k, 1)
        bytes_it = float(n) * n * A_dev.element_size() * (3 if pre else 1)
        gbs = bytes_it / per_it / 1e9
        out[name] = {"converged": bool(ok), "iters": k, "relres": rel, "true_relres": true_rel,
                     "seconds": round(t, 4), "ms_per_iter": round(per_it * 1e3, 4),
                     "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                                  "alg_bytes_per_iter": bytes_it}}
    del A64
    if out["cg"]["converged"] and out["pcg_X"]["converged"]:
        out["cg_over_pcg_seconds"] = round(out["cg"]["seconds"] / out["pcg_X"]["seconds"], 2)
    m = min(cpu_n, n)
    Ac = np.asarray(A32[:m, :m], np.float64)
    rng = np.random.default_rng(seed)
    Mc = rng.standard_normal((m, m)) / m
    Mc = Mc @ Mc.T + np.eye(m)  # an SPD stand-in: the oracle's cost does not depend on M's values
    t0 = time.perf_counter()
    P.pcg(Ac, rng.standard_normal(m), M=Mc, iters=cpu_iters)
    t_cpu = time.perf_counter() - t0
    out["cpu_oracle"] = {"ms_per_iter": round(t_cpu / cpu_iters * 1e3, 3), "kind": "oracle",
                         "sample": f"{cpu_iters} oracle PCG iterations (dense M) at n={m}"}
    return out


def time_to_tolerance(A_dev, A32, q, seed, tol, max_iters, torch, rbfgs, pcg=True):
    """AdaRBFGS (Gaussian sketch) from L_0 = I to ||I - AX||_F / sqrt(n) <= tol, mixed and
    FP64 on the same A; wall time includes every estimator read and exact residual check.
    The mixed run's X then preconditions CG on the same A."""
    out = {}
    for prec in ("mixed", "fp64"):
        A = A_dev if prec == "mixed" else A_dev.to(torch.float64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with rbfgs.Solver(A, q, seed, sketch="gauss", variant="adaptive", precision=prec) as s:
            ok, iters, resid = s.invert(tol, max_iters)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if prec == "mixed" and pcg:
                out["pcg"] = pcg_section(s, A_dev, A32, seed, torch)
        out[prec] = {"converged": bool(ok), "iters": iters, "resid": resid, "seconds": round(t, 3)}
        del A
    if out["mixed"]["converged"] and out["fp64"]["converged"]:
        out["fp64_over_mixed"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 2)
    out["tol"] = tol
    # fixed RBFGS (mixed) on the same A: with coordinates to the tolerance; with the Gaussian
    # sketch it stalls far above it on this kappa ~ 1e6 matrix, so it runs to a short cap and
    # reports the residual reached
    for name, sk, cap in (("fixed_coord", "coord", 20000), ("fixed_gauss", "gauss", 3000)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with rbfgs.Solver(A_dev, q, seed, sketch=sk, variant="fixed", precision="mixed") as s:
            ok, iters, resid = s.invert(tol, cap)
            if not ok:
                resid = s.residual() / math.sqrt(A_dev.shape[0])
        torch.cuda.synchronize()
        out[name] = {"converged": bool(ok), "iters": iters, "resid": resid, "cap": cap,
                     "seconds": round(time.perf_counter() - t0, 3)}
    return out


def sampling_section(A_dev, A32, q, seed, torch, rbfgs, tol=1e-3, cap=4000, steps=20, cpu_n=2048):
    """AdaRBFGS (mixed) on the same matrix with three sketch distributions: Gaussian,
    uniform coordinates, and the partition of Sec. 9.3 drawn with the probabilities of
    eq. ihsih0 (q divides n): iters/s over `steps` timed iterations, the phases of the
    partition run (the draw and the O(nq) weight update, with the weight kernel's HBM
    roofline: it reads the two n x q FP32 panels and reads and writes the n FP64
    weights), and the time to ||I - AX||_F / sqrt(n) <= tol from L_0 = I.  The oracle's
    partition AdaRBFGS iteration (its weights from the definition, n^3 per iteration) is
    timed at n = cpu_n."""
    import numpy as np
    from oracle import partition as Pt
    n = A_dev.shape[0]
    out = {"tol": tol}
    for sk in ("gauss", "coord", "partition"):
        row = {}
        s, dt, _ = timed_steps(rbfgs.Solver, A_dev, q, seed, sk, "adaptive", "mixed", 3, steps, torch)
        row["iters_per_s"] = round(steps / dt, 2)
        if sk == "partition":
            s.profile(1)
            s.step(10)
            rep = s.profile_report()
            s.profile(0)
            ph = {k: v[0] / max(v[1], 1) for k, v in rep.items()}
            row["phases_ms"] = {k: round(v, 4) for k, v in ph.items()}
            if ph.get("weights"):
                nbytes = 2.0 * n * q * 4 + 16.0 * n
                gbs = nbytes / (ph["weights"] * 1e-3) / 1e9
                row["weights_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                                           "alg_bytes_per_launch": nbytes}
        s.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with rbfgs.Solver(A_dev, q, seed, sketch=sk, variant="adaptive", precision="mixed") as s2:
            ok, iters, resid = s2.invert(tol, cap)
        torch.cuda.synchronize()
        row.update({"converged": bool(ok), "iters": iters, "resid": resid,
                    "seconds": round(time.perf_counter() - t0, 3)})
        out[sk] = row
    m = max(q, min(cpu_n, n) // q * q)
    Ac = np.asarray(A32[:m, :m], np.float64)
    t0 = time.perf_counter()
    Pt.run_ada(Ac, q, seed, 2)
    t_cpu = (time.perf_counter() - t0) / 2
    out["cpu_oracle"] = {"value": round(1.0 / t_cpu, 3), "unit": "iters/s", "kind": "oracle",
                         "sample": f"2 oracle partition AdaRBFGS iterations at n={m}, q={q} (leading block of A)"}
    return out


def importance_section(A_dev, A32, q, seed, torch, rbfgs, steps=10, iters=100, cpu_n=1024):
    """Simultaneous randomized Kaczmarz (W = I) on the same matrix with uniform coordinate
    blocks and with the importance probabilities of eq. discoptprob taking X_k in place of
    A^-1 (mixed): iters/s over `steps` timed iterations, the exact ||I - AX||_F / sqrt(n)
    after `iters` iterations from X_0 = I, and for the importance run the phase that forms
    the weights against the FP64 MFMA peak: r symmetric q x q Grams of q rows of X^T, whose
    q (q + 1) / 2 distinct entries take 2 n flops each, n^2 (q + 1) flops in all.
    The oracle's importance iteration (weights from the definition) is timed at n = cpu_n."""
    import numpy as np
    from oracle import partition as Pt
    n = A_dev.shape[0]
    out = {"iters": iters}
    for sk in ("coord", "importance"):
        row = {}
        s, dt, _ = timed_steps(rbfgs.Solver, A_dev, q, seed, sk, "kaczmarz", "mixed", 2, steps, torch)
        row["iters_per_s"] = round(steps / dt, 2)
        if sk == "importance":
            s.profile(1)
            s.step(3)
            rep = s.profile_report()
            s.profile(0)
            ph = {k: v[0] / max(v[1], 1) for k, v in rep.items()}
            row["phases_ms"] = {k: round(v, 4) for k, v in ph.items()}
            if ph.get("importance"):
                flops = float(n) * n * (q + 1)
                tf = flops / (ph["importance"] * 1e-3) / 1e12
                row["weights_roofline"] = {"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                                           "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                                           "traffic": None, "alg_flops": flops}
        s.close()
        with rbfgs.Solver(A_dev, q, seed, sketch=sk, variant="kaczmarz", precision="mixed") as s2:
            s2.step(iters)
            row["resid_after"] = s2.residual() / math.sqrt(n)
        out[sk] = row
    m = max(q, min(cpu_n, n) // q * q)
    Ac = np.asarray(A32[:m, :m], np.float64)
    t0 = time.perf_counter()
    Pt.run_kaczmarz_importance(Ac, q, seed, 2)
    t_cpu = (time.perf_counter() - t0) / 2
    out["cpu_oracle"] = {"value": round(1.0 / t_cpu, 3), "unit": "iters/s", "kind": "oracle",
                         "sample": f"2 oracle importance Kaczmarz iterations at n={m}, q={q} (leading block of A)"}
    return out


SPLIT_PASSES = {"XY": 3, "AS": 3, "update": 3}  # bf16 piece products issued per product (mixed, fixed/Gaussian)


def c4_section(qs, seed, torch, rbfgs, steps=200, warmup=3, samples=4096):
    """n = 32768: A = Q diag(lambda) Q^T with Q a product of 64 seeded Householder reflectors
    (compact WY in FP64 on the host, stored FP32: 4 GiB), lambda log-uniform in [1e-2, 1e2];
    fixed RBFGS, Gaussian sketch, mixed precision, `steps` timed iterations per q after
    `warmup`, the n x n product kernels timed live with HIP events.  Per q and kernel: HBM
    GB/s of algorithmic bytes, algorithmic TFLOP/s (2 n^2 q per product, the symmetric update
    on its triangle) and issued TFLOP/s (the split-bf16 piece products) against the bf16
    MFMA peak.  q = 32 sits below the ridge point (HBM-bound), q = 512 above it once the split
    passes are counted.  The error is that of 4096 sampled entries of X against the exact
    A^-1 of the same construction (with 1/lambda)."""
    import numpy as np
    from workloads import householder_entries, householder_spd
    n = 32768
    t0 = time.perf_counter()
    A = householder_spd(n, seed)
    A_dev = torch.from_numpy(A).cuda()
    del A
    torch.cuda.synchronize()
    out = {"n": n, "steps": steps, "input_gen_s": round(time.perf_counter() - t0, 1)}
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, n, samples)
    cols = rng.integers(0, n, samples)
    exact = householder_entries(n, seed, rows, cols, inverse=True)
    ri = torch.from_numpy(rows).cuda()
    ci = torch.from_numpy(cols).cuda()
    for q in qs:
        s, dt, live = timed_steps(rbfgs.Solver, A_dev, q, seed, "gauss", "fixed", "mixed", warmup, steps, torch,
                                  events=True)
        X = s.x()
        got = X[ri, ci].cpu().numpy()
        del X
        s.close()
        kern = {}
        for ph in ("XY", "AS", "update"):
            if ph not in live:
                continue
            avg = live[ph][0] / live[ph][1] / 1e3
            nbytes = phase_roofline(ph, n, q, "fixed", "gauss")[1]
            flops = 2.0 * n * n * q
            kern[ph] = {"avg_ms": round(avg * 1e3, 4), "hbm_gbs": round(nbytes / avg / 1e9, 1),
                        "alg_tflops": round(flops / avg / 1e12, 1),
                        "issued_tflops": round(SPLIT_PASSES[ph] * flops / avg / 1e12, 1),
                        "issued_mfma_frac": round(SPLIT_PASSES[ph] * flops / avg / 1e12 / BF16_PEAK_TFLOPS, 4)}
        dom = max(kern, key=lambda k: kern[k]["avg_ms"])
        bound = "hbm" if q <= 256 else "mfma"
        if bound == "hbm":
            ach, peak, unit = kern[dom]["hbm_gbs"], HBM_PEAK_GBS, "GB/s"
        else:
            ach, peak, unit = kern[dom]["alg_tflops"], BF16_PEAK_TFLOPS, "TFLOP/s"
        out[f"q{q}"] = {"value": round(steps / dt, 2), "unit": "iters/s", "ms_per_step": round(dt / steps * 1e3, 3),
                        "tflops_effective": round(alg_flops(n, q, "fixed", "gauss") * steps / dt / 1e12, 1),
                        "roofline": {"bound": bound, "kernel": dom, "achieved": ach, "peak": peak, "unit": unit,
                                     "frac": round(ach / peak, 4), "traffic": None},
                        "kernels": kern,
                        "sampled_rel_err_vs_exact_inverse": float(np.linalg.norm(got - exact) / np.linalg.norm(exact))}
    del A_dev
    return out


def live_roofline(live, n, q, variant, sketch, traffic=None):
    """Roofline object of the dominant n x n product kernel (largest total live time)."""
    products = {k: v for k, v in live.items() if phase_roofline(k, n, q, variant, sketch)}
    dominant = max(products, key=lambda k: products[k][0], default=None)
    if not dominant:
        return None
    bound, units, unit = phase_roofline(dominant, n, q, variant, sketch)
    avg_s = products[dominant][0] / products[dominant][1] / 1e3
    achieved = units / avg_s / 1e9
    tr = traffic(dominant) if traffic else None
    return {"bound": bound, "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": unit, "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None if tr is None else round(tr),
            "launches": products[dominant][1], "avg_ms": round(avg_s * 1e3, 4), "alg_bytes_per_launch": units}


def variants_section(A_dev, A32, q, seed, sketch, warmup, steps, torch, rbfgs):
    """PSB, AIP and simultaneous randomized Kaczmarz on the same matrix (the ridge Hessian
    is symmetric positive definite, so all three apply): mixed iters/s with the dominant
    kernel's live roofline, the FP64 oracle timed on one iteration beside it, and the
    one-iteration parity of the GPU iterate (mixed and FP64) against that oracle step."""
    import numpy as np
    from oracle import sketch as sk, variants as V
    n = A32.shape[0]
    A64 = np.asarray(A32, dtype=np.float64)
    S0 = sk.sketch(seed, 0, n, q, "cols" if sketch == "coord" else "gauss")
    out = {}
    for v in ("psb", "aip", "kaczmarz"):
        sv, dtv, live = timed_steps(rbfgs.Solver, A_dev, q, seed, sketch, v, "mixed", warmup, steps, torch,
                                    events=True)
        sv.close()
        ips = steps / dtv
        t0 = time.perf_counter()
        Xo = V.STEPS[v](np.eye(n), A64, S0)
        t_or = time.perf_counter() - t0
        par = {}
        for prec in ("mixed", "fp64"):
            Ause = A_dev if prec == "mixed" else A_dev.to(torch.float64)
            with rbfgs.Solver(Ause, q, seed, sketch=sketch, variant=v, precision=prec) as s:
                s.step(1)
                Xg = s.x().cpu().numpy()
            par[prec] = float(np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo))
            del Xg
        del Xo
        flops = alg_flops(n, q, v, sketch)
        out[v] = {"value": round(ips, 3), "unit": "iters/s", "ms_per_step": round(dtv / steps * 1e3, 4),
                  "steps": steps, "tflops_effective": round(flops * ips / 1e12, 3),
                  "roofline": live_roofline(live, n, q, v, sketch),
                  "products_ms_timed_region": {k: round(x[0] / max(x[1], 1), 4) for k, x in live.items()},
                  "cpu_oracle": {"value": round(1.0 / t_or, 4), "unit": "iters/s",
                                 "sample": f"1 FP64 oracle iteration from X_0 = I (n={n}, q={q})"},
                  "parity_1_step_rel_fro_err": par}
    return out


def experiment1(sizes, seed, torch, rbfgs):
    """Sec. 10, Experiment 1, on synthetic matrices: A = M^T M with M uniform on [0, 1)
    (a matrix built from rand; formed in FP64 on the GPU), q = floor(sqrt(n)).  Each method
    runs from its own starting point (AdaRBFGS: X_0 = I; Newton-Schulz: 0.99 A^T / rho^2(A);
    MR: the projected identity) until ||I - A X_k||_F / ||I - A X_0||_F < 1e-2.  The time
    includes creating the context and computing X_0 (as the paper's does), not the
    matrix; ||I - A X_0||_F is taken beforehand in an untimed context.  Newton-Schulz and
    MR are FP64 only; AdaRBFGS runs in both precisions.  The FP64 oracle's per-iteration
    time at the smallest n is reported beside."""
    import numpy as np
    from oracle import comparison as Cm, rbfgs as R, sketch as sk
    out = {}
    runs = [("adarbfgs_gauss", "adaptive", "gauss", "fp64"), ("adarbfgs_gauss_mixed", "adaptive", "gauss", "mixed"),
            ("adarbfgs_cols", "adaptive", "coord", "fp64"), ("newton_schulz", "newton_schulz", "gauss", "fp64"),
            ("mr", "mr", "gauss", "fp64")]
    for n in sizes:
        g = torch.Generator(device="cuda").manual_seed(seed + n)
        M = torch.rand((n, n), generator=g, device="cuda", dtype=torch.float64)
        A64 = M.T @ M
        del M
        A32 = A64.to(torch.float32)
        A64 = A32.to(torch.float64)  # both precisions invert the same (FP32-representable) matrix
        torch.cuda.synchronize()
        q = int(math.isqrt(n))
        row = {"q": q}
        for name, variant, sketch, prec in runs:
            Ause = A32 if prec == "mixed" else A64
            cap = 20000 if variant == "adaptive" else 300
            with rbfgs.Solver(Ause, q, seed, sketch=sketch, variant=variant, precision=prec) as s0:
                r0 = s0.residual()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with rbfgs.Solver(Ause, q, seed, sketch=sketch, variant=variant, precision=prec,
                              check_every=4 if variant == "adaptive" else 1) as s:
                ok, iters, resid = s.invert(tol=1e-2 * r0 / math.sqrt(n), max_iters=cap)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            row[name] = {"seconds": round(t, 4), "iters": int(iters), "reached": bool(ok),
                         "rel_err": round(resid * math.sqrt(n) / r0, 5)}
        # the comparison methods' iterations against the FP64 MFMA roofline: Newton-Schulz
        # forms A X and X (A X) (4 n^3 flops), MR A X, X R and R R (6 n^3)
        for meth, nprod in (("newton_schulz", 2), ("mr", 3)):
            s, dt, _ = timed_steps(rbfgs.Solver, A64, q, seed, "gauss", meth, "fp64", 1, 5, torch)
            s.close()
            tf = 2.0 * nprod * float(n) ** 3 * 5 / dt / 1e12
            row[meth]["iter_ms"] = round(dt / 5 * 1e3, 3)
            row[meth]["roofline"] = {"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4), "traffic": None}
        out[str(n)] = row
        del A32, A64
    # the oracle's time per iteration at the smallest n (FP64, host cores)
    n = sizes[0]
    g = torch.Generator(device="cuda").manual_seed(seed + n)
    M = torch.rand((n, n), generator=g, device="cuda", dtype=torch.float64)
    A = (M.T @ M).to(torch.float32).to(torch.float64).cpu().numpy()
    q = int(math.isqrt(n))
    per = {}
    t0 = time.perf_counter()
    L = np.eye(n)
    for k in range(3):
        L = R.ada_step(L, A, sk.sketch(seed, k, n, q, "gauss"))
    per["adarbfgs_gauss"] = round((time.perf_counter() - t0) / 3, 5)
    for meth in ("newton_schulz", "mr"):
        t0 = time.perf_counter()
        Cm.run(meth, A, 3)
        per[meth] = round((time.perf_counter() - t0) / 3, 5)
    out["cpu_oracle_s_per_iter"] = {"n": n, "s_per_iter": per, "kind": "oracle"}
    return out


def c1_curve(torch, rbfgs, n=256, q=16, steps=300, seed=1, every=25):
    """The n = 256 FP64 workload (A = Q diag(lambda) Q^T, lambda log-uniform in [1, 1e3], seeded
    Gaussian Q), fixed RBFGS with a Gaussian q = 16 sketch from X_0 = I: ||I - A X_k||_F (the
    library's exact FP64 residual) and ||X_k - A^-1||_F (A^-1 in closed form) after every step,
    beside the same two quantities along the FP64 oracle's trajectory."""
    import numpy as np
    from oracle import rbfgs as R
    from workloads import spectral_spd
    A, Ainv = spectral_spd(n, seed, 1.0, 1e3)
    gres, gerr = [], []
    t0 = time.perf_counter()
    with rbfgs.Solver(torch.from_numpy(A).cuda(), q, seed, precision="fp64") as s:
        for _ in range(steps):
            s.step(1)
            gres.append(s.residual())
            gerr.append(float(np.linalg.norm(s.x().cpu().numpy() - Ainv)))
    t_gpu = time.perf_counter() - t0
    ores, oerr = [], []
    R.run_fixed(A, q, seed, "gauss", steps,
                record=lambda k, X: (ores.append(R.residual_fro(A, X)), oerr.append(float(np.linalg.norm(X - Ainv)))))
    gres, gerr, ores, oerr = map(np.array, (gres, gerr, ores, oerr))
    at = [1] + list(range(every, steps + 1, every))
    return {"workload": f"spectral SPD n={n}, lambda in [1, 1e3], fixed RBFGS gauss q={q}, FP64, X_0 = I",
            "steps_logged": at,
            "resid_fro": [float(f"{gres[k - 1]:.5g}") for k in at],
            "err_vs_inverse_fro": [float(f"{gerr[k - 1]:.5g}") for k in at],
            "resid0_fro": float(np.linalg.norm(np.eye(n) - A)),
            "max_rel_dev_vs_oracle": {"resid": float(np.max(np.abs(gres - ores) / ores)),
                                      "err": float(np.max(np.abs(gerr - oerr) / oerr))},
            "gpu_s_incl_per_step_checks": round(t_gpu, 3)}


def host_info():
    """CPU model, logical CPUs, BLAS threads and RAM of the host the oracle runs on."""
    info = {"cpu_model": None, "logical_cpus": os.cpu_count(), "ram_gib": None}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    info["openblas_num_threads"] = os.environ.get("OPENBLAS_NUM_THREADS")
    return info


def cpu_baseline(A32, q, seed, sketch, variant, steps):
    """The FP64 oracle on the host: `steps` iterations from X_0 = I (or L_0 = I)."""
    import numpy as np
    from oracle import rbfgs as R, sketch as sk
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    A = np.asarray(A32, dtype=np.float64)
    n = A.shape[0]
    kind = "cols" if sketch == "coord" else "gauss"
    M = np.eye(n)
    t0 = time.perf_counter()
    for k in range(steps):
        S = sk.sketch(seed, k, n, q, kind)
        M = R.fixed_step(M, A, S) if variant == "fixed" else R.ada_step(M, A, S)
    t = time.perf_counter() - t0
    X = M if variant == "fixed" else M @ M.T
    return steps / t, threads, X


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--q", type=int, default=256)
    ap.add_argument("--seed", type=int, default=2016)
    ap.add_argument("--variant", default="fixed", choices=["fixed", "adaptive"])
    ap.add_argument("--sketch", default="gauss", choices=["gauss", "coord"])
    ap.add_argument("--fp64-steps", type=int, default=8)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-steps", type=int, default=4, help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--exp1-sizes", default="1000,2000,5000",
                    help="sizes of the Experiment-1 comparison (AdaRBFGS vs Newton-Schulz vs MR; empty: skip)")
    ap.add_argument("--variant-steps", type=int, default=20,
                    help="timed iterations of each of PSB, AIP and Kaczmarz (0: skip them)")
    ap.add_argument("--ttt-iters", type=int, default=4000,
                    help="iteration cap of the AdaRBFGS time-to-tolerance runs (0: skip them)")
    ap.add_argument("--sampling-iters", type=int, default=4000,
                    help="iteration cap of the AdaRBFGS sketch-distribution comparison (0: skip it)")
    ap.add_argument("--importance-iters", type=int, default=100,
                    help="Kaczmarz iterations of the importance-sampling comparison (0: skip it)")
    ap.add_argument("--c4-qs", default="32,512",
                    help="sketch sizes of the n = 32768 Householder runs (bandwidth- and MFMA-bound; empty: skip)")
    ap.add_argument("--c4-steps", type=int, default=200)
    ap.add_argument("--c1-steps", type=int, default=300, help="steps of the n = 256 per-step curve (0: skip)")
    ap.add_argument("--serve-jobs", type=int, default=512, help="serving trace length (0: skip serving)")
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-tol", type=float, default=1e-3)
    ap.add_argument("--serve-baseline", type=int, default=1, help="also serve the trace one at a time in FP64")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the sharded row-block "
                                   "design is described, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1602_01768_amd import rbfgs

    dev = "cuda"
    n, q = args.n, args.q
    t_gen = time.perf_counter()
    A_dev, A32, ridge_info = make_A(n, args.seed, torch, rbfgs)
    t_gen = time.perf_counter() - t_gen
    A64_dev = A_dev.to(torch.float64)
    torch.cuda.synchronize()

    # ---- timed region: mixed precision; the product kernels timed live with HIP events
    log("timed region")
    s_mixed, dt, live = timed_steps(rbfgs.Solver, A_dev, q, args.seed, args.sketch, args.variant, "mixed",
                                    args.warmup, args.steps, torch, events=True)
    ips = args.steps / dt
    flops = alg_flops(n, q, args.variant, args.sketch)
    roof = live_roofline(live, n, q, args.variant, args.sketch,
                         counter_traffic if args.sketch == "gauss" and args.variant == "fixed" else None)
    live_ms = {k: round(v[0] / max(v[1], 1), 4) for k, v in live.items()}

    # ---- all phases timed in a separate window (informational)
    log("all phases timed in a separate window (informational)")
    s_mixed.profile(1)
    s_mixed.step(args.profile_steps)
    rep = s_mixed.profile_report()
    s_mixed.profile(0)
    phases = {k: {"avg_ms": v[0] / max(v[1], 1), "count": v[1]} for k, v in rep.items()}
    s_mixed.close()

    # ---- FP64 GPU path on the same matrix
    log("FP64 GPU path on the same matrix")
    s64, dt64, _ = timed_steps(rbfgs.Solver, A64_dev, q, args.seed, args.sketch, args.variant, "fp64", 1,
                               args.fp64_steps, torch)
    ips64 = args.fp64_steps / dt64
    s64.close()
    del A64_dev

    # ---- AdaRBFGS (the method that reaches the tolerance on this workload), mixed, same timing
    log("AdaRBFGS (the method that reaches the tolerance on this work")
    s_ada, dt_ada, live_ada = timed_steps(rbfgs.Solver, A_dev, q, args.seed, "gauss", "adaptive", "mixed",
                                          args.warmup, args.steps, torch, events=True)
    s_ada.close()
    ada_flops = alg_flops(n, q, "adaptive", "gauss")
    adaptive = {"value": round(args.steps / dt_ada, 3), "unit": "iters/s",
                "ms_per_step": round(dt_ada / args.steps * 1e3, 4),
                "tflops_effective": round(ada_flops * args.steps / dt_ada / 1e12, 3),
                "products_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in live_ada.items()},
                "roofline": live_roofline(live_ada, n, q, "adaptive", "gauss", lambda p: counter_traffic("ada." + p))}

    # ---- the other instances of the family (PSB, AIP, Kaczmarz) on the same matrix
    log("the other instances of the family (PSB, AIP, Kaczmarz) on th")
    variants = (variants_section(A_dev, A32, q, args.seed, args.sketch, args.warmup, args.variant_steps, torch, rbfgs)
                if args.variant_steps > 0 else None)

    # ---- Experiment 1 of Sec. 10: AdaRBFGS against Newton-Schulz and MR
    log("Experiment 1 of Sec. 10")
    sizes = [int(x) for x in args.exp1_sizes.split(",") if x.strip()]
    exp1 = experiment1(sizes, args.seed, torch, rbfgs) if sizes else None

    # ---- time to tolerance, AdaRBFGS mixed vs FP64; its X as a CG preconditioner
    log("time to tolerance, AdaRBFGS mixed vs FP64")
    ttt = (time_to_tolerance(A_dev, A32, q, args.seed, 1e-3, args.ttt_iters, torch, rbfgs)
           if args.ttt_iters > 0 else None)

    # ---- sketch distributions for AdaRBFGS: Gaussian, uniform coordinates, partition (eq. ihsih0)
    log("sketch distributions for AdaRBFGS")
    sampling = (sampling_section(A_dev, A32, q, args.seed, torch, rbfgs, cap=args.sampling_iters)
                if args.sampling_iters > 0 and n % q == 0 else None)

    # ---- Kaczmarz with importance probabilities (eq. discoptprob, X_k as the proxy)
    log("Kaczmarz with importance probabilities (eq. discoptprob, X_k")
    importance = (importance_section(A_dev, A32, q, args.seed, torch, rbfgs, iters=args.importance_iters)
                  if args.importance_iters > 0 and n % q == 0 else None)

    # ---- n = 32768 Householder matrix, q = 32 (HBM-bound) and q = 512 (MFMA-bound)
    log("n = 32768 Householder matrix, q = 32 (HBM-bound) and q = 512")
    c4_qs = [int(x) for x in args.c4_qs.split(",") if x.strip()]
    c4 = c4_section(c4_qs, args.seed, torch, rbfgs, steps=args.c4_steps) if c4_qs else None

    # ---- n = 256 FP64: ||I - A X_k||_F and ||X_k - A^-1||_F after every step, GPU beside the oracle
    log("n = 256 FP64")
    c1 = c1_curve(torch, rbfgs, steps=args.c1_steps) if args.c1_steps > 0 else None

    # ---- serving trace (p50 / p99 solve latency)
    log("serving trace (p50 / p99 solve latency)")
    serve = serving(args, torch, rbfgs) if args.serve_jobs > 0 else None

    # ---- CPU oracle baseline (bounded sample) and parity of the same steps
    log("CPU oracle baseline (bounded sample) and parity of the same ")
    cpu = None
    parity = None
    if args.cpu_steps > 0:
        A_ref = reference_A(n, args.seed, torch)
        ref_diff = float((A_ref - A_dev).abs().max() / A_dev.abs().max())
        A_ref32 = A_ref.cpu().numpy()
        cps, threads, Xo = cpu_baseline(A_ref32, q, args.seed, args.sketch, args.variant, args.cpu_steps)
        cpu = {"value": round(cps, 4), "unit": "iters/s", "cores": threads, "kind": "oracle",
               "sample": f"{args.cpu_steps} FP64 oracle iterations from X_0 = I on the same A (n={n}, q={q})",
               "host": host_info()}
        parity = {"input": "A formed by torch's FP64 GEMM from the same B (not by the library)",
                  "input_max_rel_diff_vs_library_A": ref_diff}
        for prec in ("mixed", "fp64"):
            Ause = A_ref if prec == "mixed" else A_ref.to(torch.float64)
            with rbfgs.Solver(Ause, q, args.seed, sketch=args.sketch, variant=args.variant, precision=prec) as s:
                s.step(args.cpu_steps)
                Xg = s.x().cpu().numpy()
            err = float(np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo))
            parity[prec] = {"steps": args.cpu_steps, "rel_fro_err_vs_oracle": err}
            del Xg, Ause
        del A_ref

    # the long sections first and the headline figures last, so that a reader of the line's
    # tail sees value, fp64, roofline, cpu_baseline and parity
    out = {
        "ridge_hessian": ridge_info,
        "variants": variants,
        "experiment1": exp1,
        "time_to_tolerance_ada": ttt,
        "sampling_ada": sampling,
        "importance_kaczmarz": importance,
        "c4_householder_n32768": c4,
        "serving": serve,
        "c1_curve_n256": c1,
        "phases_ms": {k: round(v["avg_ms"], 4) for k, v in phases.items()},
        "products_ms_timed_region": live_ms,
        "input_gen_s": round(t_gen, 1),
        "metric": "RBFGS iters/s + TFLOP/s (n=16384,q=256) mixed vs FP64; p50/p99 solve latency",
        "value": round(ips, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-split/f32 (f64 q x q)",
        "data": "synthetic",
        "config": {"workload": f"ridge Hessian B^T B/m + 1e-2 I, n={n}, m={2 * n}, q={q}, "
                               f"{args.variant} RBFGS, {args.sketch} sketch, seed={args.seed}",
                   "n": n, "q": q, "variant": args.variant, "sketch": args.sketch, "precision": "mixed"},
        "tflops_effective": round(flops * ips / 1e12, 3),
        "alg_flops_per_step": flops,
        "fp64": {"value": round(ips64, 3), "unit": "iters/s", "ms_per_step": round(dt64 / args.fp64_steps * 1e3, 3),
                 "tflops_effective": round(flops * ips64 / 1e12, 3), "steps": args.fp64_steps},
        "mixed_over_fp64_per_step": round(ips / ips64, 3),
        "adaptive_mixed": adaptive,
        "ada_time_to_tol_s": ({"mixed": ttt["mixed"]["seconds"], "fp64": ttt["fp64"]["seconds"],
                               "ratio": ttt.get("fp64_over_mixed")} if ttt else None),
        "serving_p50_p99_ms": ({"sojourn": [serve["mixed"]["sojourn_p50_ms"], serve["mixed"]["sojourn_p99_ms"]],
                                "rate_jobs_per_s": serve.get("arrival_rate_jobs_per_s")}
                               if serve and "mixed" in serve else None),
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
