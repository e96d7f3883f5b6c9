/*
 * rbfgs.h -- C ABI of an MI355X (gfx950) library for randomized block BFGS
 * matrix inversion: Gower & Richtarik, "Randomized Quasi-Newton Updates are
 * Linearly Convergent Matrix Inversion Algorithms" (arXiv 1602.01768).
 *
 * Problem (Sec. 4, inverse equation AX = I; Sec. 5, symmetric iterates): given a
 * symmetric positive definite A in R^{n x n}, a sketch size q and a seed, return
 * X ~ A^-1.  Two methods:
 *
 *   RBFGS_FIXED     randomized block BFGS, Sec. 8.7 eq. (qunac):
 *                   X+ = S G^-1 S^T + (I - S G^-1 S^T A) X (I - A S G^-1 S^T),
 *                   G = S^T A S, with a fresh i.i.d. sketch S every iteration.
 *   RBFGS_ADAPTIVE  AdaRBFGS, Sec. 9.3 Alg. 4 / eq. (Cholimprov): X = L L^T,
 *                   S = L S~ with S~ i.i.d.; L+ = L + S R (C S~^T - R^T S^T A L),
 *                   R = L_G^-T (G = L_G L_G^T), C = L_M^-1 (S~^T S~ = L_M L_M^T).
 *
 * Other instances of the sketch-and-project family (same sketches and stream):
 *   RBFGS_PSB       randomized Powell-symmetric-Broyden, Sec. 8.4: Alg. 3 with
 *                   W = I, read through eq. (Xupdatesym) (the printed eq. (PSB)
 *                   has garbled transposes): with Y = A S, G = Y^T Y,
 *                   X+ = X - (X A - I) S G^-1 Y^T + Y G^-1 (Y^T X - S^T)(Y G^-1 Y^T - I).
 *                   A symmetric (not necessarily definite); X stays symmetric.
 *   RBFGS_AIP       approximate inverse preconditioning, Sec. 8.6 eq. (BFGSas):
 *                   Alg. 1 with W = A^-1, X+ = X + S (S^T A S)^-1 S^T (I - A X).
 *                   A SPD; the iterates are not symmetric.
 *   RBFGS_KACZMARZ  simultaneous randomized Kaczmarz, Sec. 8.2 eq. (badbroyadj):
 *                   Alg. 1 with W = I, X+ = X + A^T S (S^T A A^T S)^-1 S^T (I - A X).
 *                   Any invertible A (row-major, not required to be symmetric).
 * The two comparison methods of Sec. 10 (FP64 only; sketch and q unused):
 *   RBFGS_NEWTON_SCHULZ  eq. (Newton-Schulz), X+ = 2X - X A X, from X_0 = 0.99 A^T / rho^2(A)
 *                   with rho(A) ~ ||A||_2 by 100 power-method steps from the all-ones vector;
 *   RBFGS_MR        eq. (MRiter), X+ = X + alpha X R, R = I - A X,
 *                   alpha = Tr(R^T A X R) / Tr((A X R)^T A X R), from X_0 = (Tr A / Tr(A A^T)) I.
 *   Their estimator is the exact ||I - A X_k||_F^2 of the iterate each step starts from.
 * For PSB, AIP and Kaczmarz a coordinate sketch is applied as the dense 0/1 matrix,
 * and the estimator of AIP and Kaczmarz is ||S^T (I - A X)||_F^2 scaled as for the
 * fixed method (it estimates ||I - A X||_F^2).
 *
 * Sketch distributions (Sec. 10): RBFGS_SKETCH_GAUSS, S~ n x q with i.i.d.
 * N(0,1) entries; RBFGS_SKETCH_COORD, q distinct coordinate vectors drawn
 * uniformly.  Both come from a counter-based stream keyed by (seed, iteration),
 * so a run is reproducible bit for bit and can be resumed from (X_k, k):
 *   key = (seed, 0), counter = (block, k, kind, 0), Philox4x64-10;
 *   gauss: entry e = j*n + i uses block e>>2, word e&3, Box-Muller pairs on
 *          words (0,1), (2,3) with u = ((x>>11)+0.5) 2^-53, rounded to 8
 *          significant bits (bfloat16 values) nearest-even;
 *   coord: Floyd's algorithm with Lemire's bounded draws on the word stream,
 *          indices sorted ascending.
 * RBFGS_SKETCH_PARTITION (fixed RBFGS and AdaRBFGS; q must divide n): S~ = I_{:C_i} for
 * the block C_i = [iq, (i+1)q) of a partition of [n], drawn with the probabilities of
 * eq. (ihsih0), p_i = Tr(S_i^T A S_i) / Tr(S^T A S) -- the complete discrete sampling
 * that the convergence results of Sec. 7.3 and Sec. 9.3 assume.  Fixed RBFGS: S_i =
 * I_{:C_i}, weights the diagonal of A.  AdaRBFGS: S_i = L_k I_{:C_i}, weights the
 * diagonal of L_k^T A L_k, kept on the device in O(nq) per step through
 * L+^T A L+ = L^T A L - K K^T + S~ (S~^T S~)^-1 S~^T, K = L^T A S R, and recomputed
 * (n^3 flops) by rbfgs_set_state.  Draw: word 0 of block 0 of the kind-3 stream gives
 * u = ((x>>11)+0.5) 2^-53; the first block whose running weight sum exceeds u times the
 * total is taken.  The estimator carries the factor 1/p_i (unbiased, Horvitz-Thompson).
 * RBFGS_SKETCH_IMPORTANCE (Kaczmarz only; q must divide n): the same partition and draw,
 * with the probabilities of eq. (discoptprob) for W = I, S = I, taking the iterate X_k in
 * place of the unknown A^-1 (the heuristic of Sec. 7.2, not covered by the convergence
 * theory): p_i proportional to ||X_k I_{:C_i} I_{C_i:} A||_F = <(X_k^T X_k)_{C_i C_i},
 * (A A^T)_{C_i C_i}>^(1/2), recomputed from X_k at every iteration in FP64 (one launch over
 * all r = n/q blocks: the distinct entries of their symmetric q x q Grams of q rows, n^2 (q+1)
 * flops per step; the blocks of A A^T once at creation).  The draw needs X_k, so the
 * iteration's lanes run one step at a time (no look-ahead).
 *
 * Starting point: X_0 = I, L_0 = I (the experiments' choice, Sec. 10).
 *
 * Precision (rbfgs_precision):
 *   RBFGS_FP64   every step in FP64 on the GPU.
 *   RBFGS_MIXED  A and X (or L) stored in FP32; the n x n x q contractions and
 *                the n^2 update run on bf16 MFMA with FP32 accumulation, each
 *                FP32 operand presented as a split bf16 pair (hi + lo; A as
 *                hi + mid + lo when S is an exact bf16 matrix).  G = S^T A S, its
 *                Cholesky factor and the q x q triangular inverses, and the
 *                residual ||I - AX||_F are FP64.
 *
 * Conventions for every call:
 *   - Matrices are dense, row-major with a leading dimension (for symmetric A
 *     and X the distinction is moot; L is general and row-major).
 *   - Device pointers are HIP device addresses on the context's device;
 *     host pointers are ordinary host memory.
 *   - No call allocates memory owned by the caller; outputs go to caller
 *     buffers.  The context owns all of its device memory.
 *   - Calls return an rbfgs_status; no C++ exception crosses the ABI.  Kernel
 *     detected failures (G not positive definite, non-finite values) are
 *     recorded on the device and returned by the next call that synchronises.
 *   - A context is bound to the HIP stream given at creation and is not
 *     thread safe; distinct contexts may be used from distinct threads.
 *   - Results are deterministic: the same (A, params) on the same device and
 *     build gives bitwise identical iterates.
 */
#ifndef RBFGS_H
#define RBFGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbfgs_ctx rbfgs_ctx;

typedef enum {
  RBFGS_OK = 0,
  RBFGS_E_INVALID_ARG = 1,   /* bad size, pointer, enum, or A not symmetric/finite */
  RBFGS_E_OOM = 2,           /* device allocation failed */
  RBFGS_E_NOT_SPD = 3,       /* Cholesky of G = S^T A S (or S~^T S~) met a pivot <= 0 */
  RBFGS_E_NONFINITE = 4,     /* NaN/Inf appeared in the iteration */
  RBFGS_E_NOT_CONVERGED = 5, /* rbfgs_invert hit max_iters above tolerance */
  RBFGS_E_DEVICE = 6,        /* a HIP runtime call failed */
  RBFGS_E_CANCELLED = 7      /* a served job was cancelled (rbfgs_server_cancel) */
} rbfgs_status;

typedef enum {
  RBFGS_SKETCH_GAUSS = 0,
  RBFGS_SKETCH_COORD = 1,
  RBFGS_SKETCH_PARTITION = 2,
  RBFGS_SKETCH_IMPORTANCE = 3
} rbfgs_sketch;
typedef enum {
  RBFGS_FIXED = 0,
  RBFGS_ADAPTIVE = 1,
  RBFGS_PSB = 2,
  RBFGS_AIP = 3,
  RBFGS_KACZMARZ = 4,
  RBFGS_NEWTON_SCHULZ = 5,
  RBFGS_MR = 6
} rbfgs_variant;
typedef enum { RBFGS_FP64 = 0, RBFGS_MIXED = 1 } rbfgs_precision;
typedef enum { RBFGS_F32 = 0, RBFGS_F64 = 1 } rbfgs_dtype;

typedef struct {
  int64_t n;            /* matrix order, n >= 1 */
  int32_t q;            /* sketch size, 1 <= q <= min(n, 1024) */
  uint64_t seed;        /* sketch stream key */
  int32_t sketch;       /* rbfgs_sketch */
  int32_t variant;      /* rbfgs_variant */
  int32_t precision;    /* rbfgs_precision */
  int32_t check_every;  /* rbfgs_invert: iterations between estimator reads (>= 1; 0 = 16) */
} rbfgs_params;

/* Create a context: validate params, copy A into library-owned device memory
 * (converted to FP32 in mixed mode, FP64 in FP64 mode), set X_0 = I (L_0 = I).
 *   A          n x n matrix, row-major, leading dimension lda >= n, element type
 *              a_dtype; host memory if a_on_device == 0, else device memory.
 *              Must be symmetric (checked exactly on the stored type; not for
 *              RBFGS_KACZMARZ) and finite; positive definiteness (where the
 *              variant needs it) is detected during iteration.
 *   hip_stream hipStream_t to run on (NULL = the default stream).
 *   out        receives the context; set to NULL on failure.
 * Errors: E_INVALID_ARG (sizes, NULL pointers, asymmetric or non-finite A),
 *         E_OOM, E_DEVICE. */
rbfgs_status rbfgs_create(const rbfgs_params* params, const void* A, int32_t a_dtype,
                          int64_t lda, int32_t a_on_device, void* hip_stream,
                          rbfgs_ctx** out);

/* Enqueue `nsteps` iterations k -> k+1 (Alg. 3 with W = A^-1, or Alg. 4) on the
 * context's stream.  Asynchronous: returns once the work is enqueued; a
 * device-side failure of these steps is returned by the next synchronising
 * call (rbfgs_sync, rbfgs_invert, rbfgs_residual, rbfgs_get_x).  After such a
 * failure the iterate is undefined: call rbfgs_set_state or re-create. */
rbfgs_status rbfgs_step(rbfgs_ctx* ctx, int64_t nsteps);

/* Wait for enqueued work; return the first device-side failure, if any. */
rbfgs_status rbfgs_sync(rbfgs_ctx* ctx);

/* Iterate until ||I - A X_k||_F / sqrt(n) <= tol or max_iters total iterations
 * (Sec. 10 stops on a residual threshold).  Every check_every iterations the mean
 * of the window's per-step unbiased estimates of ||I - X A||_F^2 (from S - X A S, no
 * extra products; for the adaptive method they estimate ||I - L^T A L||_F^2) is read;
 * when it falls below the trigger (tol^2 n, lowered by the ratio estimate / exact
 * residual^2 observed at each failed check) the exact FP64 residual is computed and
 * decides.  For AdaRBFGS, whose free estimate measures ||I - L^T A L||_F^2 (a lower
 * bound of ||I - A X||_F^2), the trigger is instead an unbiased FP64 estimate of
 * ||I - A X||_F^2 from 64 Gaussian probe vectors (6 n^2 64 flops), taken only when the
 * window mean is below tol^2 n, must fall below 0.8 tol^2 n.  A check is also forced after max(64 check_every,
 * iterations so far) iterations without one (AdaRBFGS: 256 check_every; coordinate and
 * partition sketches of the fixed method, whose estimates are heavy-tailed: max(16
 * check_every, half the iterations so far)).
 * iters_out: iterations performed by this call; resid_out: last exact
 * ||I - AX||_F / sqrt(n) (NaN if never computed).  Either may be NULL.
 * Returns OK on convergence, E_NOT_CONVERGED at max_iters, or a device error. */
rbfgs_status rbfgs_invert(rbfgs_ctx* ctx, double tol, int64_t max_iters,
                          int64_t* iters_out, double* resid_out);

/* Exact ||I - A X_k||_F (unnormalised) in FP64 on the device (X = L L^T for the
 * adaptive method); synchronises. */
rbfgs_status rbfgs_residual(rbfgs_ctx* ctx, double* fro_out);

/* Last per-step estimator value sum||S - XAS||^2 scaled to estimate ||I-XA||_F^2
 * (gauss: /q, coord: *n/q); synchronises. NaN before the first step. */
rbfgs_status rbfgs_estimate(rbfgs_ctx* ctx, double* est_out);

/* Copy X_k (X = L L^T formed in FP64 for the adaptive method) into X, row-major,
 * leading dimension ldx >= n, element type x_dtype, host or device memory.
 * Synchronises. */
rbfgs_status rbfgs_get_x(rbfgs_ctx* ctx, void* X, int32_t x_dtype, int64_t ldx,
                         int32_t on_device);

/* Copy the factor L_k of the adaptive method (E_INVALID_ARG for the fixed one). */
rbfgs_status rbfgs_get_l(rbfgs_ctx* ctx, void* L, int32_t l_dtype, int64_t ldl,
                         int32_t on_device);

/* Replace the state by (M, k): M is X_k for the fixed method, L_k for the
 * adaptive one (row-major, leading dimension ldm, element type m_dtype, host
 * or device).  Used for checkpoint/resume: the sketch of iteration k depends
 * only on (seed, k), so resuming reproduces the uninterrupted run.  The
 * iterates of the fixed method and PSB are symmetric, and M must be too (not
 * checked): the steps may read an entry from either triangle. */
rbfgs_status rbfgs_set_state(rbfgs_ctx* ctx, const void* M, int32_t m_dtype, int64_t ldm,
                             int32_t on_device, int64_t k);

/* Partition sampling: copy the n per-coordinate FP64 weights (the diagonal of A for
 * fixed RBFGS, of L_k^T A L_k for AdaRBFGS; for importance sampling the weight of each
 * block on its first coordinate, zeros elsewhere, as of the last draw) to host memory;
 * synchronises.  E_INVALID_ARG unless the context samples partitions. */
rbfgs_status rbfgs_get_weights(rbfgs_ctx* ctx, double* out);

/* Iterations performed so far (k of X_k). */
rbfgs_status rbfgs_get_iter(const rbfgs_ctx* ctx, int64_t* k_out);

/* Release all device memory of the context (waits for its stream). NULL is a no-op. */
void rbfgs_destroy(rbfgs_ctx* ctx);

/* Human-readable description of the last error on ctx ("" if none).  The
 * string is owned by the context and valid until the next call on it. */
const char* rbfgs_last_error(const rbfgs_ctx* ctx);

/* ---- timing of the iteration's phases (tracing aid) ----
 * rbfgs_profile: per-phase timing of subsequent iterations with HIP events
 * recorded on the stream each phase runs on, and clear the accumulated totals.
 * enable = 0 off, 1 every phase, 2 only the n x n products (AS, XY, LS, LtY,
 * update: the fewest events, for timing inside a measured run); other values
 * E_INVALID_ARG.  Phases: sketch, sample, importance, sketch_gram, gather, AS, LS, gram_G, chol_inv,
 * panel_U, XY, LtY, gram_H, estimator, panels (containing weights), coord_update, update; a split-K
 * product also reports its reduction kernel as "<phase>.reduce", so that the
 * phase itself times the product kernel alone.
 * rbfgs_profile_report: synchronise and write a JSON object
 * {"phase": [total_ms, count], ...} (NUL-terminated) into buf of buflen bytes;
 * E_INVALID_ARG if it does not fit. */
rbfgs_status rbfgs_profile(rbfgs_ctx* ctx, int32_t enable);
rbfgs_status rbfgs_profile_report(rbfgs_ctx* ctx, char* buf, int64_t buflen);

/* Solve A x = b by conjugate gradients preconditioned with the context's current
 * approximate inverse -- the use of X ~ A^-1 that motivates the method (Sec. 1):
 * textbook PCG (Hestenes & Stiefel; Saad, Alg. 9.1) from x_0 = 0 with z = M r,
 * M = X_k (fixed RBFGS) or L_k L_k^T applied as L (L^T r) (AdaRBFGS) when precond = 1,
 * M = I (plain CG) when precond = 0.  FP64 vectors; A and X as the context stores them.
 * Stops when ||r_k|| <= tol ||b|| (tested every 8 iterations) or after max_iters.
 *   b, x   n-vectors of b_dtype / x_dtype (F32 or F64), host or device memory.
 *   iters_out, relres_out: iterations run and the last ||r_k|| / ||b|| (may be NULL).
 * Needs an SPD A (not PSB, Kaczmarz) and, with precond = 1, a fixed or adaptive context.
 * Allocates O(n) work memory of its own; synchronises.  Returns OK, E_NOT_CONVERGED,
 * E_NONFINITE, E_INVALID_ARG or a device error. */
rbfgs_status rbfgs_pcg(rbfgs_ctx* ctx, const void* b, int32_t b_dtype, int32_t b_on_device, void* x, int32_t x_dtype,
                       int32_t x_on_device, int32_t precond, double tol, int64_t max_iters, int64_t* iters_out,
                       double* relres_out);

/* Ridge-regression Hessian, eq. (ridgeMatrix): A = scale * B^T B + lambda I for an
 * m x n data matrix B (the benchmark's workload takes scale = 1/m), in FP64 on the
 * GPU (FP64 MFMA, the symmetric product on lower tiles mirrored, so A is exactly
 * symmetric), then rounded to a_dtype.
 *   B   m x n row-major, leading dimension ldb >= n, element type b_dtype; host or
 *       device memory (b_on_device).
 *   A   n x n row-major output, leading dimension lda >= n, element type a_dtype;
 *       host or device memory (a_on_device).
 * Allocates and frees its own FP64 work buffers (about 8 (m n + n^2) bytes after
 * padding); synchronises the stream before returning.
 * Errors: E_INVALID_ARG (sizes, pointers, non-finite scale or lambda), E_OOM, E_DEVICE. */
rbfgs_status rbfgs_ridge_hessian(const void* B, int32_t b_dtype, int64_t m, int64_t n, int64_t ldb,
                                 int32_t b_on_device, double scale, double lambda, void* A, int32_t a_dtype,
                                 int64_t lda, int32_t a_on_device, void* hip_stream);

/* For callers that cannot allocate device memory -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc: rbfgs_ridge_hessian for device-resident B
 * and A, which allocates and frees nothing and does not synchronise (asynchronous on
 * hip_stream, whose device must be the current device).  Its work buffers -- B copied to
 * FP64 with rows padded to mp = 16 ceil(m/16) and columns to np = 128 ceil(n/128), the
 * np x np FP64 product and two scalars -- live in a fixed device array of
 * RBFGS_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends; they are cleared by fill kernels (no memset nodes when captured).
 *   Limit: 8 (mp np + np np) + 256 <= RBFGS_NOALLOC_SCRATCH_BYTES (for n <= 1024: m <= 7152).
 *   Arguments as for rbfgs_ridge_hessian; B and A are device pointers.
 * All calls on one GPU share that GPU's array and leave it holding the last call's buffers:
 * calls whose work overlaps on one GPU (different streams, or host threads without an
 * ordering between their streams) race; serialise them, e.g. on one stream.
 * Errors: E_INVALID_ARG (sizes beyond the limit, bad sizes, pointers, non-finite scale or
 * lambda), E_DEVICE (a launch failed or the array's address could not be obtained). */
#define RBFGS_NOALLOC_SCRATCH_BYTES (64ull << 20)
rbfgs_status rbfgs_ridge_hessian_noalloc(const void* B, int32_t b_dtype, int64_t m, int64_t n, int64_t ldb,
                                         double scale, double lambda, void* A, int32_t a_dtype, int64_t lda,
                                         void* hip_stream);

/* ---- sketch stream (Sec. 10 sketch distributions), for testing and reuse ----
 * Write the iteration-k sketch of the stream (seed) to device memory on `hip_stream`.
 *   rbfgs_sketch_gauss: S n x q column-major (entry (i,j) at S[j*n + i]) as
 *                       float (dtype F32) or double (F64); values are bfloat16.
 *   rbfgs_sketch_coord: q sorted distinct int32 indices in [0, n).
 * Asynchronous; E_INVALID_ARG for bad sizes/pointers. */
rbfgs_status rbfgs_sketch_gauss(uint64_t seed, int64_t k, int64_t n, int32_t q,
                                void* S_dev, int32_t dtype, void* hip_stream);
rbfgs_status rbfgs_sketch_coord(uint64_t seed, int64_t k, int64_t n, int32_t q,
                                int32_t* idx_dev, void* hip_stream);

/* Partition draw of iteration k (RBFGS_SKETCH_PARTITION): block i of the partition of
 * [0, n) into consecutive blocks C_i = [iq, (i+1)q) with probability w_i / sum_j w_j,
 * w_i = max(0, sum_{c in C_i} t[c]) (eq. ihsih0 when t is the diagonal of A, or of
 * L^T A L).  t_dev: n FP64 weights on the device.  Writes idx_dev[0..q) = C_i and, when
 * ht_dev is not NULL, ht_dev[0] = 1/p_i.  A weight total that is not finite and positive
 * draws block 0 (with ht 1).  Asynchronous on hip_stream; E_INVALID_ARG unless q
 * divides n (1 <= q <= n <= 2^20) and the pointers are set. */
rbfgs_status rbfgs_sample_partition(const double* t_dev, int64_t n, int32_t q, uint64_t seed, int64_t k,
                                    int32_t* idx_dev, double* ht_dev, void* hip_stream);

/* Device bytes a context for `params` holds (plus, for the adaptive method, the
 * n x n FP64 scratch of its exact residual), computed without allocating.  Used by
 * the server's admission control.  E_INVALID_ARG for invalid sizes. */
rbfgs_status rbfgs_footprint(const rbfgs_params* params, int64_t* bytes_out);

/* ---- serving: many inversions (Sec. 10 stopping rule) sharing one GPU ----
 * Continuous batching under one scheduler thread.  The server allocates one device-memory
 * pool of budget_bytes when it starts; every job's context takes its buffers from it, so
 * admitting and retiring a job allocates and frees no device memory.  Jobs are admitted first
 * come, first served, into a slot table of `workers` slots when a slot is free and the job's
 * footprint (rbfgs_footprint) fits the pool beside the running jobs.  Each slot has a stream
 * (at most 4 streams in all; slots beyond 4 share them round-robin), on which the job's
 * context runs all of its lanes; the job advances in windows of check_every iterations, each
 * followed by the stopping decision of rbfgs_invert.  Windows are enqueued without blocking
 * the host -- the scheduler polls their events -- so the windows of all resident jobs are on
 * the GPU together.  With the Gaussian sketch (fixed RBFGS or AdaRBFGS) and check_every a
 * multiple of 3, a job's full windows are one HIP graph, captured at its first window and
 * replayed (the sketch's iteration then comes from a device counter).  A job's iterates,
 * iteration count and residual are those of rbfgs_invert on the job alone.  Times are seconds
 * on a monotonic clock started at rbfgs_server_create.  The server is thread-safe; calls from
 * several host threads may interleave. */
typedef struct rbfgs_server rbfgs_server;

typedef struct {
  uint64_t tag;      /* the caller's job tag */
  int32_t status;    /* rbfgs_status of the job (OK: converged to tol) */
  int64_t iters;     /* iterations run */
  double resid;      /* last exact ||I - AX||_F / sqrt(n) (NaN if never computed) */
  double t_submit;   /* submission */
  double t_admit;    /* admission into a slot */
  double t_done;     /* completion */
} rbfgs_job_result;

typedef struct {
  double now;            /* server clock */
  int64_t queued;        /* submitted, not started */
  int32_t running;       /* in a slot now */
  int64_t outstanding;   /* queued + running */
  int64_t active_bytes;  /* footprints of the running jobs */
  int64_t peak_bytes;    /* largest active_bytes so far (<= budget) */
  int32_t peak_running;  /* most jobs running at once so far */
} rbfgs_server_info;

/* workers (slots) in [1, 64], budget_bytes > 0 (the pool, allocated here).  E_INVALID_ARG,
 * E_OOM (the pool could not be allocated), E_DEVICE. */
rbfgs_status rbfgs_server_create(int64_t budget_bytes, int32_t workers, rbfgs_server** out);

/* Queue one inversion: A as in rbfgs_create (it must stay valid and unchanged until
 * the job's result has been polled), iterate with rbfgs_invert(tol, max_iters);
 * when x_out != NULL copy X_k there at the end (as rbfgs_get_x; also when not
 * converged).  Returns at once: E_INVALID_ARG for invalid arguments (as
 * rbfgs_create, plus tol <= 0, max_iters < 0), E_OOM when the job alone exceeds the
 * budget; every other outcome arrives in the job's result. */
rbfgs_status rbfgs_server_submit(rbfgs_server* server, const rbfgs_params* params, const void* A,
                                 int32_t a_dtype, int64_t lda, int32_t a_on_device, double tol,
                                 int64_t max_iters, void* x_out, int32_t x_dtype, int64_t ldx,
                                 int32_t x_on_device, uint64_t tag);

/* Move up to max_results finished jobs (in completion order) into results; *n_out
 * receives the count.  If none is ready and jobs are outstanding, wait up to
 * wait_ms milliseconds for one. */
rbfgs_status rbfgs_server_poll(rbfgs_server* server, rbfgs_job_result* results, int32_t max_results,
                               int32_t* n_out, int32_t wait_ms);

/* Cancel the earliest outstanding job carrying `tag`.  A job still queued is removed and its
 * result (status E_CANCELLED, 0 iterations) is posted at once.  A running job stops at its next
 * window boundary -- the window in flight completes, no further one is enqueued -- and its
 * result carries E_CANCELLED, the iterations run and, when x_out was given, X_k as for a job
 * that did not converge; its memory returns to the pool.  A job that finishes on its own before
 * the request is seen keeps its own status.  E_INVALID_ARG when no outstanding job carries the
 * tag (or every running one already has a request pending). */
rbfgs_status rbfgs_server_cancel(rbfgs_server* server, uint64_t tag);

/* Snapshot of the queue and the budget use. */
rbfgs_status rbfgs_server_stats(rbfgs_server* server, rbfgs_server_info* info);

/* Finish every submitted job, then stop the workers and free the server;
 * results not yet polled are discarded. */
void rbfgs_server_destroy(rbfgs_server* server);

#ifdef __cplusplus
}
#endif

#endif /* RBFGS_H */
