// C ABI of the RBFGS library: context management and the per-iteration
// orchestration of the kernels.  See include/rbfgs.h for the contract.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "../../include/rbfgs.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace rb;

struct rbfgs_ctx {
  rbfgs_params p{};
  int64_t n = 0, np = 0, qp = 0;
  int q = 0;
  bool mixed = false, ada = false, coord = false;
  int mdt = DT_F64;  // element type of A, X/L and the n x q panels
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t k = 0;
  std::string err;
  // device buffers
  void* A = nullptr;
  void* X = nullptr;        // X (fixed) or L (adaptive)
  void* Sk = nullptr;       // sketch (S, or S~ for the adaptive method); bf16 in mixed mode
  int32_t* C = nullptr;     // coordinate indices
  int32_t* pos = nullptr;   // inverse map of C (-1 elsewhere)
  void* Sa = nullptr;       // adaptive: S = L S~
  void* Y = nullptr;
  void* V = nullptr;        // V = X Y (fixed) or T^T = L^T Y (adaptive)
  void* U = nullptr;        // fixed: U = S G^-1 (mixed) / panel [U | W' | U] (FP64)
  void* W = nullptr;        // fixed: W' (mixed); adaptive: Q^T
  __bf16* planes = nullptr; // mixed: bf16 hi/lo planes of the update operands
  void* R = nullptr;        // fixed coordinate: R = G^-1 W'^T (qp x np)
  double *G = nullptr, *H = nullptr, *Ginv = nullptr, *Z = nullptr, *GH = nullptr, *Zm = nullptr,
         *Mm = nullptr, *Mq = nullptr;
  double* cwork = nullptr;
  void* partial = nullptr;
  size_t partial_bytes = 0;
  double* red = nullptr;
  int64_t red_count = 0;
  double* est = nullptr;
  int* status = nullptr;
  std::vector<void*> allocs;
  // per-phase timing with HIP events on the context's stream (rbfgs_profile)
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
  };
  bool prof = false;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  std::map<std::string, std::pair<double, int64_t>> prof_acc;
};

namespace {

struct Fail {
  rbfgs_status st;
};

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                      \
      throw Fail{e_ == hipErrorOutOfMemory ? RBFGS_E_OOM : RBFGS_E_DEVICE};              \
    }                                                                                    \
  } while (0)

size_t dt_size(int dt) { return dt == DT_F32 ? 4 : (dt == DT_BF16 ? 2 : 8); }

void* dalloc(rbfgs_ctx* ctx, size_t bytes) {
  void* p = nullptr;
  HIPCHK(hipMalloc(&p, bytes ? bytes : 16));
  ctx->allocs.push_back(p);
  HIPCHK(hipMemsetAsync(p, 0, bytes ? bytes : 16, ctx->stream));
  return p;
}

hipEvent_t prof_event(rbfgs_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

// Scope that brackets the kernels of one phase of an iteration with events.
struct Phase {
  rbfgs_ctx* ctx;
  const char* name;
  hipEvent_t a = nullptr;
  Phase(rbfgs_ctx* c, const char* n) : ctx(c), name(n) {
    if (ctx->prof) {
      a = prof_event(ctx);
      HIPCHK(hipEventRecord(a, ctx->stream));
    }
  }
  ~Phase() {
    if (!ctx->prof || !a) return;
    hipEvent_t b = nullptr;
    if (!ctx->ev_pool.empty()) {
      b = ctx->ev_pool.back();
      ctx->ev_pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
      return;
    }
    if (hipEventRecord(b, ctx->stream) == hipSuccess) ctx->prof_pending.push_back({name, a, b});
  }
};

void prof_flush(rbfgs_ctx* ctx) {
  if (ctx->prof_pending.empty()) return;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (auto& r : ctx->prof_pending) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    auto& acc = ctx->prof_acc[r.name];
    acc.first += ms;
    acc.second += 1;
    ctx->ev_pool.push_back(r.a);
    ctx->ev_pool.push_back(r.b);
  }
  ctx->prof_pending.clear();
}

int pick_split(int64_t tiles, int64_t K, int kmul) {
  int s = 1;
  while (s < 8 && tiles * s < 1024 && K % ((int64_t)kmul * s * 2) == 0 && K / (s * 2) >= 256) s *= 2;
  return s;
}

int64_t f64_tile(int64_t x) { return x % 128 == 0 ? 128 : 32; }
int64_t bf_bn(int64_t N) { return N % 256 == 0 ? 256 : (N % 128 == 0 ? 128 : (N % 64 == 0 ? 64 : 32)); }

// C(M x N, col-major, ldc) = Aop * Bop in FP64 (tall-skinny or q x q products).
void f64_gemm(rbfgs_ctx* ctx, GemmArgs g) {
  if (g.epi == EPI_COLSTORE) {
    const int64_t tiles = (g.M / f64_tile(g.M)) * (g.N / f64_tile(g.N));
    g.splitk = pick_split(tiles, g.K, 16);
    const size_t need = (size_t)g.splitk * g.M * g.N * sizeof(double);
    if (g.splitk > 1 && need > ctx->partial_bytes) g.splitk = 1;
  }
  HIPCHK(gemm_f64(g, ctx->partial, ctx->stream));
}

// C(M x N, col-major float, ldc) = Aop * Bop on bf16 MFMA pieces.
void bf_gemm(rbfgs_ctx* ctx, MixedGemm mg) {
  GemmArgs& g = mg.g;
  if (g.epi == EPI_COLSTORE) {
    const int64_t tiles = (g.M / 128) * (g.N / bf_bn(g.N));
    g.splitk = pick_split(tiles, g.K, 32);
    const size_t need = (size_t)g.splitk * g.M * g.N * sizeof(float);
    if (need > ctx->partial_bytes) g.splitk = 1;
  }
  HIPCHK(gemm_bf16(mg, ctx->partial, ctx->stream));
}

// out = M * P for an n x n matrix M (A, X or L) and an n x q panel P, per precision.
// transpose: Aop = M^T (T^T = L^T Y).  In mixed mode (na, nb, pmax) choose the bf16
// pieces of each operand and the passes kept (all piece pairs with i + j <= pmax).
void nn_times_panel(rbfgs_ctx* ctx, const void* M, bool transpose, const void* P, int p_dt, void* out, int na = 2,
                    int nb = 2, int pmax = 1) {
  if (ctx->mixed) {
    MixedGemm mg;
    GemmArgs& g = mg.g;
    g.M = ctx->np; g.N = ctx->qp; g.K = ctx->np;
    g.A = M; g.lda = ctx->np;
    g.B = P; g.ldb = ctx->np;
    g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->np; g.c2 = 1.0;
    mg.a_kind = transpose ? OK_F32_MC : OK_F32_KC;
    mg.b_kind = p_dt == DT_BF16 ? OK_BF16_KC : OK_F32_KC;
    mg.na = na; mg.nb = p_dt == DT_BF16 ? 1 : nb; mg.pmax = pmax;
    bf_gemm(ctx, mg);
  } else {
    GemmArgs g;
    g.M = ctx->np; g.N = ctx->qp; g.K = ctx->np;
    g.A = M; g.lda = ctx->np; g.a_dt = DT_F64; g.a_kc = !transpose;
    g.B = P; g.ldb = ctx->np; g.b_dt = p_dt; g.b_kc = true;
    g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->np; g.c_dt = DT_F64; g.c2 = 1.0;
    f64_gemm(ctx, g);
  }
}

// q x q Gram C = P1^T P2 of two n x q column-major panels, FP64 accumulation.
void gram(rbfgs_ctx* ctx, const void* P1, int dt1, const void* P2, int dt2, double* out) {
  GemmArgs g;
  g.M = ctx->qp; g.N = ctx->qp; g.K = ctx->np;
  g.A = P1; g.lda = ctx->np; g.a_dt = dt1; g.a_kc = true;
  g.B = P2; g.ldb = ctx->np; g.b_dt = dt2; g.b_kc = true;
  g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->qp; g.c_dt = DT_F64; g.c2 = 1.0;
  f64_gemm(ctx, g);
}

// out(n x q) = c2 * P(n x q, col-major) * M(q x q, row-major) [+ c0*B0 + c1*B1]
void panel_times_small(rbfgs_ctx* ctx, const void* P, int p_dt, const double* M, void* out, int out_dt, double c2,
                       const void* B0 = nullptr, int b0_dt = DT_F64, double c0 = 0, const void* B1 = nullptr,
                       int b1_dt = DT_F64, double c1 = 0) {
  GemmArgs g;
  g.M = ctx->np; g.N = ctx->qp; g.K = ctx->qp;
  g.A = P; g.lda = ctx->np; g.a_dt = p_dt; g.a_kc = false;
  g.B = M; g.ldb = ctx->qp; g.b_dt = DT_F64; g.b_kc = false;
  g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->np; g.c_dt = out_dt; g.c2 = c2;
  g.B0 = B0; g.b0_dt = b0_dt; g.c0 = c0; g.B1 = B1; g.b1_dt = b1_dt; g.c1 = c1; g.ld01 = ctx->np;
  f64_gemm(ctx, g);
}

// out(q x q, row-major) = Aop * Bop with row-major q x q inputs (transposes by flag).
void small_small(rbfgs_ctx* ctx, const double* A, bool at, const double* B, double* out) {
  GemmArgs g;
  g.M = ctx->qp; g.N = ctx->qp; g.K = ctx->qp;
  g.A = A; g.lda = ctx->qp; g.a_dt = DT_F64; g.a_kc = !at;
  g.B = B; g.ldb = ctx->qp; g.b_dt = DT_F64; g.b_kc = false;
  g.epi = EPI_ROWSTORE; g.C = out; g.ldc = ctx->qp; g.c_dt = DT_F64; g.c2 = 1.0;
  f64_gemm(ctx, g);
}

void do_sketch(rbfgs_ctx* ctx, int64_t k) {
  if (ctx->coord) {
    HIPCHK(sketch_coord(ctx->p.seed, k, ctx->n, ctx->q, ctx->C, ctx->stream));
  } else {
    HIPCHK(sketch_gauss(ctx->p.seed, k, ctx->n, ctx->q, ctx->Sk, ctx->mixed ? DT_BF16 : DT_F64, ctx->np,
                        ctx->stream));
  }
}

int sk_dt(const rbfgs_ctx* ctx) { return ctx->mixed ? DT_BF16 : DT_F64; }

// One fixed-sketch RBFGS iteration, eq. (qunac) as the symmetric rank-2q update
//   X+ = X - (U W'^T + W' U^T),  U = S G^-1,  W' = V - S/2 - U H/2,
//   Y = A S,  G = S^T Y,  V = X Y,  H = Y^T V.
void step_fixed(rbfgs_ctx* ctx) {
  const int64_t np = ctx->np, qp = ctx->qp;
  const int mdt = ctx->mdt;
  { Phase ph(ctx, "sketch"); do_sketch(ctx, ctx->k); }
  if (ctx->coord) {
    Phase ph(ctx, "gather");
    HIPCHK(gather_cols_sym(ctx->A, mdt, np, ctx->C, ctx->q, np, ctx->Y, mdt, np, ctx->G, qp, ctx->stream));
  } else {
    { Phase ph(ctx, "AS"); nn_times_panel(ctx, ctx->A, false, ctx->Sk, sk_dt(ctx), ctx->Y, 3, 1, 2); }  // exact products
    Phase ph(ctx, "gram_G");
    gram(ctx, ctx->Sk, sk_dt(ctx), ctx->Y, mdt, ctx->G);
  }
  { Phase ph(ctx, "chol_inv"); HIPCHK(chol_inv(ctx->G, qp, ctx->q, ctx->Z, ctx->Ginv, qp, ctx->cwork, ctx->status, ctx->stream)); }
  { Phase ph(ctx, "XY"); nn_times_panel(ctx, ctx->X, false, ctx->Y, mdt, ctx->V); }
  { Phase ph(ctx, "gram_H"); gram(ctx, ctx->Y, mdt, ctx->V, mdt, ctx->H); }
  const double scale = ctx->coord ? (double)ctx->n / ctx->q : 1.0 / ctx->q;
  {
    Phase ph(ctx, "estimator");
    HIPCHK(estimator(ctx->coord ? nullptr : ctx->Sk, sk_dt(ctx), ctx->coord ? ctx->C : nullptr, ctx->V, mdt, np,
                     ctx->n, ctx->q, scale, ctx->red, ctx->est, ctx->status, ctx->stream));
  }
  if (ctx->coord) {
    Phase ph(ctx, "coord_update");
    // U = E_C G^-1 is not formed: W' = V - E_C/2 - E_C (G^-1 H)/2 and R = G^-1 W'^T;
    // the update touches only rows and columns C.
    small_small(ctx, ctx->Ginv, false, ctx->H, ctx->GH);
    HIPCHK(hipMemcpyAsync(ctx->W, ctx->V, (size_t)np * qp * dt_size(mdt), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(coord_wprime_fix(ctx->W, mdt, np, ctx->C, ctx->q, ctx->GH, qp, ctx->stream));
    GemmArgs g;
    g.M = qp; g.N = np; g.K = qp;
    g.A = ctx->Ginv; g.lda = qp; g.a_dt = DT_F64; g.a_kc = true;
    g.B = ctx->W; g.ldb = np; g.b_dt = mdt; g.b_kc = false;
    g.epi = EPI_ROWSTORE; g.C = ctx->R; g.ldc = np; g.c_dt = mdt; g.c2 = 1.0;
    f64_gemm(ctx, g);
    HIPCHK(coord_sym_update(ctx->X, mdt, np, ctx->C, ctx->pos, ctx->q, np, ctx->R, mdt, np, ctx->stream));
    return;
  }
  if (ctx->mixed) {
    float* U = (float*)ctx->U;
    float* W = (float*)ctx->W;
    const int64_t ldp = 3 * qp, plane = np * ldp;  // operand planes [U | W' | U], row-major
    __bf16* hi = ctx->planes;
    __bf16* lo = ctx->planes + plane;
    {
      Phase ph(ctx, "panels");
      panel_times_small(ctx, ctx->Sk, DT_BF16, ctx->Ginv, U, DT_F32, 1.0);
      panel_times_small(ctx, U, DT_F32, ctx->H, W, DT_F32, -0.5, ctx->V, DT_F32, 1.0, ctx->Sk, DT_BF16, -0.5);
      HIPCHK(pack_split2(U, np, np, qp, hi, lo, ldp, 0, ctx->stream));
      HIPCHK(pack_split2(W, np, np, qp, hi, lo, ldp, qp, ctx->stream));
      HIPCHK(pack_split2(U, np, np, qp, hi, lo, ldp, 2 * qp, ctx->stream));
    }
    Phase ph(ctx, "update");
    MixedGemm mg;
    GemmArgs& g = mg.g;
    g.M = np; g.N = np; g.K = 2 * qp;
    g.A = hi; g.lda = ldp; g.a_plane = plane;
    g.B = hi + qp; g.ldb = ldp; g.b_plane = plane;
    g.epi = EPI_SYMUPD; g.C = ctx->X; g.ldc = np; g.c2 = -1.0;
    mg.a_kind = OK_BF16_KC; mg.b_kind = OK_BF16_KC; mg.na = 2; mg.nb = 2; mg.pmax = 1;
    bf_gemm(ctx, mg);
  } else {
    double* PQ = (double*)ctx->U;  // [U | W' | U], column-major, ld = np
    double* U = PQ;
    double* W = PQ + np * qp;
    {
      Phase ph(ctx, "panels");
      panel_times_small(ctx, ctx->Sk, DT_F64, ctx->Ginv, U, DT_F64, 1.0);
      panel_times_small(ctx, U, DT_F64, ctx->H, W, DT_F64, -0.5, ctx->V, DT_F64, 1.0, ctx->Sk, DT_F64, -0.5);
      HIPCHK(hipMemcpyAsync(PQ + 2 * np * qp, U, (size_t)np * qp * sizeof(double), hipMemcpyDeviceToDevice,
                            ctx->stream));
    }
    Phase ph(ctx, "update");
    GemmArgs g;
    g.M = np; g.N = np; g.K = 2 * qp;
    g.A = PQ; g.lda = np; g.a_dt = DT_F64; g.a_kc = false;
    g.B = PQ + np * qp; g.ldb = np; g.b_dt = DT_F64; g.b_kc = false;
    g.epi = EPI_SYMUPD; g.C = ctx->X; g.ldc = np; g.c_dt = DT_F64; g.c2 = -1.0;
    f64_gemm(ctx, g);
  }
}

// One AdaRBFGS iteration, eq. (Cholimprov) with R = L_G^-T, C = L_M^-1:
//   S = L S~,  Y = A S,  G = S^T Y = L_G L_G^T,  T^T = L^T Y,
//   Q^T = S~ (L_M^-T L_G^-1) - T^T G^-1,  L+ = L + S Q.
void step_adaptive(rbfgs_ctx* ctx) {
  const int64_t np = ctx->np, qp = ctx->qp;
  const int mdt = ctx->mdt;
  { Phase ph(ctx, "sketch"); do_sketch(ctx, ctx->k); }
  if (ctx->coord) {
    Phase ph(ctx, "gather");
    HIPCHK(gather_cols_gen(ctx->X, mdt, np, ctx->C, ctx->q, np, ctx->Sa, mdt, np, ctx->stream));
  } else {
    Phase ph(ctx, "LS");
    nn_times_panel(ctx, ctx->X, false, ctx->Sk, sk_dt(ctx), ctx->Sa, 3, 1, 2);  // S = L S~, exact products
  }
  { Phase ph(ctx, "AS"); nn_times_panel(ctx, ctx->A, false, ctx->Sa, mdt, ctx->Y, 3, 2, 2); }
  { Phase ph(ctx, "gram_G"); gram(ctx, ctx->Sa, mdt, ctx->Y, mdt, ctx->G); }
  { Phase ph(ctx, "chol_inv"); HIPCHK(chol_inv(ctx->G, qp, ctx->q, ctx->Z, ctx->Ginv, qp, ctx->cwork, ctx->status, ctx->stream)); }
  { Phase ph(ctx, "LtY"); nn_times_panel(ctx, ctx->X, true, ctx->Y, mdt, ctx->V, 2, 3, 2); }  // T^T = L^T Y
  const double scale = ctx->coord ? (double)ctx->n / ctx->q : 1.0 / ctx->q;
  {
    Phase ph(ctx, "panels");
    HIPCHK(estimator(ctx->coord ? nullptr : ctx->Sk, sk_dt(ctx), ctx->coord ? ctx->C : nullptr, ctx->V, mdt, np,
                     ctx->n, ctx->q, scale, ctx->red, ctx->est, ctx->status, ctx->stream));
    // Q^T = -T^T G^-1 (+ S~ Mq)
    panel_times_small(ctx, ctx->V, mdt, ctx->Ginv, ctx->W, mdt, -1.0);
    if (ctx->coord) {
      HIPCHK(coord_add_rows(ctx->W, mdt, np, ctx->C, ctx->q, ctx->Z, qp, ctx->stream));  // Mq = Z_G
    } else {
      gram(ctx, ctx->Sk, sk_dt(ctx), ctx->Sk, sk_dt(ctx), ctx->Mm);
      HIPCHK(chol_inv(ctx->Mm, qp, ctx->q, ctx->Zm, nullptr, qp, ctx->cwork, ctx->status, ctx->stream));
      small_small(ctx, ctx->Zm, true, ctx->Z, ctx->Mq);  // Mq = Z_M^T Z_G
      panel_times_small(ctx, ctx->Sk, sk_dt(ctx), ctx->Mq, ctx->W, mdt, 1.0, ctx->W, mdt, 1.0);
    }
  }
  // L += S Q
  Phase ph(ctx, "update");
  if (ctx->mixed) {
    const int64_t plane = np * qp;
    __bf16* shi = ctx->planes;
    __bf16* qhi = ctx->planes + 2 * plane;
    HIPCHK(pack_split2((const float*)ctx->Sa, np, np, qp, shi, shi + plane, qp, 0, ctx->stream));
    HIPCHK(pack_split2((const float*)ctx->W, np, np, qp, qhi, qhi + plane, qp, 0, ctx->stream));
    MixedGemm mg;
    GemmArgs& g = mg.g;
    g.M = np; g.N = np; g.K = qp;
    g.A = shi; g.lda = qp; g.a_plane = plane;
    g.B = qhi; g.ldb = qp; g.b_plane = plane;
    g.epi = EPI_ADDROW; g.C = ctx->X; g.ldc = np; g.c2 = 1.0;
    mg.a_kind = OK_BF16_KC; mg.b_kind = OK_BF16_KC; mg.na = 2; mg.nb = 2; mg.pmax = 1;
    bf_gemm(ctx, mg);
  } else {
    GemmArgs g;
    g.M = np; g.N = np; g.K = qp;
    g.A = ctx->Sa; g.lda = np; g.a_dt = DT_F64; g.a_kc = false;
    g.B = ctx->W; g.ldb = np; g.b_dt = DT_F64; g.b_kc = false;
    g.epi = EPI_ADDROW; g.C = ctx->X; g.ldc = np; g.c_dt = DT_F64; g.c2 = 1.0;
    f64_gemm(ctx, g);
  }
}

rbfgs_status fail(rbfgs_ctx* ctx, rbfgs_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

rbfgs_status read_status(rbfgs_ctx* ctx) {
  int st = 0;
  HIPCHK(hipMemcpyAsync(&st, ctx->status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (st == 3) return fail(ctx, RBFGS_E_NOT_SPD, "Cholesky of S^T A S met a non-positive pivot (A not SPD?)");
  if (st == 4) return fail(ctx, RBFGS_E_NONFINITE, "non-finite value in the iteration");
  if (st) return fail(ctx, RBFGS_E_DEVICE, "unknown device status");
  return RBFGS_OK;
}

double exact_residual(rbfgs_ctx* ctx) {
  const int64_t np = ctx->np;
  void* tmp = nullptr;
  GemmArgs g;
  g.M = np; g.N = np; g.K = np;
  g.A = ctx->A; g.lda = np; g.a_dt = ctx->mdt; g.a_kc = true;
  if (ctx->ada) {
    // B = A L (FP64), then I - B L^T
    HIPCHK(hipMalloc(&tmp, (size_t)np * np * sizeof(double)));
    GemmArgs b = g;
    b.B = ctx->X; b.ldb = np; b.b_dt = ctx->mdt; b.b_kc = false;
    b.epi = EPI_ROWSTORE; b.C = tmp; b.ldc = np; b.c_dt = DT_F64; b.c2 = 1.0;
    HIPCHK(gemm_f64(b, nullptr, ctx->stream));
    g.A = tmp; g.a_dt = DT_F64;
  }
  g.B = ctx->X; g.ldb = np; g.b_dt = ctx->mdt; g.b_kc = true;  // X symmetric; for L: Bop(k,j) = L[j][k]
  g.epi = EPI_RESID; g.red = ctx->red; g.nvalid = ctx->n;
  const int64_t blocks = gemm_f64_blocks(g);
  HIPCHK(gemm_f64(g, nullptr, ctx->stream));
  HIPCHK(reduce_sum(ctx->red, blocks, ctx->est + 1, ctx->stream));
  double r2 = 0;
  HIPCHK(hipMemcpyAsync(&r2, ctx->est + 1, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (tmp) HIPCHK(hipFree(tmp));
  return sqrt(r2);
}

}  // namespace

extern "C" {

rbfgs_status rbfgs_create(const rbfgs_params* params, const void* A, int32_t a_dtype, int64_t lda,
                          int32_t a_on_device, void* hip_stream, rbfgs_ctx** out) {
  if (!out) return RBFGS_E_INVALID_ARG;
  *out = nullptr;
  if (!params || !A) return RBFGS_E_INVALID_ARG;
  const rbfgs_params& p = *params;
  if (p.n < 1 || p.q < 1 || p.q > p.n || p.q > 1024 || lda < p.n || (a_dtype != RBFGS_F32 && a_dtype != RBFGS_F64) ||
      (p.sketch != RBFGS_SKETCH_GAUSS && p.sketch != RBFGS_SKETCH_COORD) ||
      (p.variant != RBFGS_FIXED && p.variant != RBFGS_ADAPTIVE) ||
      (p.precision != RBFGS_FP64 && p.precision != RBFGS_MIXED) || p.check_every < 0 || p.n > (1ll << 20))
    return RBFGS_E_INVALID_ARG;
  rbfgs_ctx* ctx = new rbfgs_ctx();
  ctx->p = p;
  if (ctx->p.check_every == 0) ctx->p.check_every = 16;
  ctx->n = p.n;
  ctx->q = p.q;
  ctx->np = (p.n + 255) / 256 * 256;
  ctx->qp = ((int64_t)p.q + 31) / 32 * 32;
  ctx->mixed = p.precision == RBFGS_MIXED;
  ctx->ada = p.variant == RBFGS_ADAPTIVE;
  ctx->coord = p.sketch == RBFGS_SKETCH_COORD;
  ctx->mdt = ctx->mixed ? DT_F32 : DT_F64;
  ctx->stream = (hipStream_t)hip_stream;
  try {
    HIPCHK(hipGetDevice(&ctx->device));
    const int64_t np = ctx->np, qp = ctx->qp;
    const size_t es = dt_size(ctx->mdt);
    ctx->A = dalloc(ctx, np * np * es);
    ctx->X = dalloc(ctx, np * np * es);
    ctx->Sk = dalloc(ctx, np * qp * dt_size(sk_dt(ctx)));
    ctx->C = (int32_t*)dalloc(ctx, qp * sizeof(int32_t));
    ctx->pos = (int32_t*)dalloc(ctx, np * sizeof(int32_t));
    HIPCHK(hipMemsetAsync(ctx->pos, 0xff, np * sizeof(int32_t), ctx->stream));  // -1
    ctx->Y = dalloc(ctx, np * qp * es);
    ctx->V = dalloc(ctx, np * qp * es);
    ctx->W = dalloc(ctx, np * qp * es);
    if (ctx->ada) ctx->Sa = dalloc(ctx, np * qp * es);
    if (!ctx->ada) ctx->U = dalloc(ctx, (ctx->mixed ? 1 : 3) * np * qp * es);
    if (ctx->mixed) ctx->planes = (__bf16*)dalloc(ctx, (size_t)2 * 3 * np * qp * sizeof(__bf16));
    if (!ctx->ada && ctx->coord) ctx->R = dalloc(ctx, qp * np * es);
    const size_t qq = (size_t)qp * qp * sizeof(double);
    ctx->G = (double*)dalloc(ctx, qq);
    ctx->H = (double*)dalloc(ctx, qq);
    ctx->Ginv = (double*)dalloc(ctx, qq);
    ctx->Z = (double*)dalloc(ctx, qq);
    ctx->GH = (double*)dalloc(ctx, qq);
    ctx->Zm = (double*)dalloc(ctx, qq);
    ctx->Mm = (double*)dalloc(ctx, qq);
    ctx->Mq = (double*)dalloc(ctx, qq);
    ctx->cwork = (double*)dalloc(ctx, chol_inv_work_doubles(ctx->q) * sizeof(double));
    ctx->partial_bytes = std::max<size_t>((size_t)8 * np * qp * es, (size_t)64 * qp * qp * sizeof(double));
    ctx->partial = dalloc(ctx, ctx->partial_bytes);
    ctx->red_count = std::max<int64_t>(4096, (np / 32) * (np / 32) + 16);
    ctx->red = (double*)dalloc(ctx, ctx->red_count * sizeof(double));
    ctx->est = (double*)dalloc(ctx, 4 * sizeof(double));
    ctx->status = (int*)dalloc(ctx, sizeof(int));
    // copy A (n x n, lda) into the padded np x np buffer, converting its type
    const int sdt = a_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
    const size_t ses = dt_size(sdt);
    const void* Adev = A;
    void* staging = nullptr;
    if (!a_on_device) {
      HIPCHK(hipMalloc(&staging, (size_t)p.n * lda * ses));
      HIPCHK(hipMemcpyAsync(staging, A, (size_t)p.n * lda * ses, hipMemcpyHostToDevice, ctx->stream));
      Adev = staging;
    }
    int* flag = ctx->status;
    HIPCHK(check_sym_finite(Adev, sdt, lda, p.n, flag, ctx->stream));
    HIPCHK(copy_convert(Adev, sdt, lda, ctx->A, ctx->mdt, np, p.n, p.n, ctx->stream));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (staging) HIPCHK(hipFree(staging));
    if (bad) {
      rbfgs_destroy(ctx);
      return RBFGS_E_INVALID_ARG;
    }
    if (ctx->mixed) {
      // the stored FP32 A must also be symmetric and finite
      HIPCHK(check_sym_finite(ctx->A, DT_F32, np, p.n, flag, ctx->stream));
      HIPCHK(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (bad) {
        rbfgs_destroy(ctx);
        return RBFGS_E_INVALID_ARG;
      }
    }
    HIPCHK(set_identity(ctx->X, ctx->mdt, np, p.n, ctx->stream));
    const double nanv = NAN;
    HIPCHK(hipMemcpyAsync(ctx->est, &nanv, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  } catch (const Fail& f) {
    rbfgs_destroy(ctx);
    return f.st;
  }
  *out = ctx;
  return RBFGS_OK;
}

rbfgs_status rbfgs_step(rbfgs_ctx* ctx, int64_t nsteps) {
  if (!ctx || nsteps < 0) return RBFGS_E_INVALID_ARG;
  try {
    for (int64_t i = 0; i < nsteps; ++i) {
      if (ctx->ada) step_adaptive(ctx);
      else step_fixed(ctx);
      ++ctx->k;
    }
  } catch (const Fail& f) {
    return f.st;
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_sync(rbfgs_ctx* ctx) {
  if (!ctx) return RBFGS_E_INVALID_ARG;
  try {
    return read_status(ctx);
  } catch (const Fail& f) {
    return f.st;
  }
}

rbfgs_status rbfgs_residual(rbfgs_ctx* ctx, double* fro_out) {
  if (!ctx || !fro_out) return RBFGS_E_INVALID_ARG;
  try {
    rbfgs_status st = read_status(ctx);
    if (st != RBFGS_OK) return st;
    *fro_out = exact_residual(ctx);
  } catch (const Fail& f) {
    return f.st;
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_estimate(rbfgs_ctx* ctx, double* est_out) {
  if (!ctx || !est_out) return RBFGS_E_INVALID_ARG;
  try {
    rbfgs_status st = read_status(ctx);
    if (st != RBFGS_OK) return st;
    HIPCHK(hipMemcpy(est_out, ctx->est, sizeof(double), hipMemcpyDeviceToHost));
  } catch (const Fail& f) {
    return f.st;
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_invert(rbfgs_ctx* ctx, double tol, int64_t max_iters, int64_t* iters_out, double* resid_out) {
  if (!ctx || !(tol > 0) || max_iters < 0) return RBFGS_E_INVALID_ARG;
  int64_t done = 0;
  double resid = NAN;
  double thresh = tol * tol * (double)ctx->n;  // estimator target for ||I - XA||_F^2
  rbfgs_status result = RBFGS_E_NOT_CONVERGED;
  try {
    while (done < max_iters) {
      const int64_t m = std::min<int64_t>(ctx->p.check_every, max_iters - done);
      rbfgs_status st = rbfgs_step(ctx, m);
      if (st != RBFGS_OK) { result = st; break; }
      done += m;
      st = read_status(ctx);
      if (st != RBFGS_OK) { result = st; break; }
      double est = 0;
      HIPCHK(hipMemcpy(&est, ctx->est, sizeof(double), hipMemcpyDeviceToHost));
      if (est <= thresh) {
        const double r = exact_residual(ctx);
        resid = r / sqrt((double)ctx->n);
        if (resid <= tol) { result = RBFGS_OK; break; }
        // the estimate runs below the exact value: scale the trigger by the observed ratio
        if (r > 0 && est > 0) thresh = std::min(thresh, tol * tol * (double)ctx->n * est / (r * r));
      }
    }
  } catch (const Fail& f) {
    result = f.st;
  }
  if (iters_out) *iters_out = done;
  if (resid_out) *resid_out = resid;
  if (result == RBFGS_E_NOT_CONVERGED) ctx->err = "max_iters reached above tolerance";
  return result;
}

static rbfgs_status copy_out(rbfgs_ctx* ctx, const void* src, int src_dt, int64_t lds, void* dst, int32_t d_dtype,
                             int64_t ldd, int32_t on_device) {
  const int ddt = d_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
  const int64_t n = ctx->n;
  if (on_device) {
    HIPCHK(copy_convert(src, src_dt, lds, dst, ddt, ldd, n, n, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RBFGS_OK;
  }
  void* tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, (size_t)n * ldd * dt_size(ddt)));
  HIPCHK(copy_convert(src, src_dt, lds, tmp, ddt, ldd, n, n, ctx->stream));
  HIPCHK(hipMemcpyAsync(dst, tmp, (size_t)n * ldd * dt_size(ddt), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipFree(tmp));
  return RBFGS_OK;
}

rbfgs_status rbfgs_get_x(rbfgs_ctx* ctx, void* X, int32_t x_dtype, int64_t ldx, int32_t on_device) {
  if (!ctx || !X || ldx < ctx->n || (x_dtype != RBFGS_F32 && x_dtype != RBFGS_F64)) return RBFGS_E_INVALID_ARG;
  try {
    rbfgs_status st = read_status(ctx);
    if (st != RBFGS_OK) return st;
    if (!ctx->ada) return copy_out(ctx, ctx->X, ctx->mdt, ctx->np, X, x_dtype, ldx, on_device);
    const int64_t np = ctx->np;
    void* tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, (size_t)np * np * sizeof(double)));
    GemmArgs g;
    g.M = np; g.N = np; g.K = np;
    g.A = ctx->X; g.lda = np; g.a_dt = ctx->mdt; g.a_kc = true;
    g.B = ctx->X; g.ldb = np; g.b_dt = ctx->mdt; g.b_kc = true;  // Bop(k,j) = L[j][k]
    g.epi = EPI_ROWSTORE; g.C = tmp; g.ldc = np; g.c_dt = DT_F64; g.c2 = 1.0;
    HIPCHK(gemm_f64(g, nullptr, ctx->stream));
    st = copy_out(ctx, tmp, DT_F64, np, X, x_dtype, ldx, on_device);
    HIPCHK(hipFree(tmp));
    return st;
  } catch (const Fail& f) {
    return f.st;
  }
}

rbfgs_status rbfgs_get_l(rbfgs_ctx* ctx, void* L, int32_t l_dtype, int64_t ldl, int32_t on_device) {
  if (!ctx || !L || !ctx->ada || ldl < ctx->n || (l_dtype != RBFGS_F32 && l_dtype != RBFGS_F64))
    return RBFGS_E_INVALID_ARG;
  try {
    rbfgs_status st = read_status(ctx);
    if (st != RBFGS_OK) return st;
    return copy_out(ctx, ctx->X, ctx->mdt, ctx->np, L, l_dtype, ldl, on_device);
  } catch (const Fail& f) {
    return f.st;
  }
}

rbfgs_status rbfgs_set_state(rbfgs_ctx* ctx, const void* M, int32_t m_dtype, int64_t ldm, int32_t on_device,
                             int64_t k) {
  if (!ctx || !M || ldm < ctx->n || k < 0 || (m_dtype != RBFGS_F32 && m_dtype != RBFGS_F64))
    return RBFGS_E_INVALID_ARG;
  try {
    const int sdt = m_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
    const int64_t n = ctx->n;
    const void* src = M;
    void* staging = nullptr;
    if (!on_device) {
      HIPCHK(hipMalloc(&staging, (size_t)n * ldm * dt_size(sdt)));
      HIPCHK(hipMemcpyAsync(staging, M, (size_t)n * ldm * dt_size(sdt), hipMemcpyHostToDevice, ctx->stream));
      src = staging;
    }
    HIPCHK(copy_convert(src, sdt, ldm, ctx->X, ctx->mdt, ctx->np, n, n, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->status, 0, sizeof(int), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (staging) HIPCHK(hipFree(staging));
    ctx->k = k;
  } catch (const Fail& f) {
    return f.st;
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_get_iter(const rbfgs_ctx* ctx, int64_t* k_out) {
  if (!ctx || !k_out) return RBFGS_E_INVALID_ARG;
  *k_out = ctx->k;
  return RBFGS_OK;
}

void rbfgs_destroy(rbfgs_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& r : ctx->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (void* p : ctx->allocs) (void)hipFree(p);
  delete ctx;
}

rbfgs_status rbfgs_profile(rbfgs_ctx* ctx, int32_t enable) {
  if (!ctx) return RBFGS_E_INVALID_ARG;
  try {
    prof_flush(ctx);
    ctx->prof_acc.clear();
  } catch (const Fail& f) {
    return f.st;
  }
  ctx->prof = enable != 0;
  return RBFGS_OK;
}

rbfgs_status rbfgs_profile_report(rbfgs_ctx* ctx, char* buf, int64_t buflen) {
  if (!ctx || !buf || buflen < 3) return RBFGS_E_INVALID_ARG;
  try {
    prof_flush(ctx);
  } catch (const Fail& f) {
    return f.st;
  }
  std::string out = "{";
  bool first = true;
  for (auto& kv : ctx->prof_acc) {
    char item[256];
    snprintf(item, sizeof(item), "%s\"%s\": [%.6f, %lld]", first ? "" : ", ", kv.first.c_str(), kv.second.first,
             (long long)kv.second.second);
    out += item;
    first = false;
  }
  out += "}";
  if ((int64_t)out.size() + 1 > buflen) return RBFGS_E_INVALID_ARG;
  memcpy(buf, out.c_str(), out.size() + 1);
  return RBFGS_OK;
}

const char* rbfgs_last_error(const rbfgs_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

rbfgs_status rbfgs_sketch_gauss(uint64_t seed, int64_t k, int64_t n, int32_t q, void* S_dev, int32_t dtype,
                                void* hip_stream) {
  if (!S_dev || n < 1 || q < 1 || k < 0 || (dtype != RBFGS_F32 && dtype != RBFGS_F64)) return RBFGS_E_INVALID_ARG;
  hipError_t e = sketch_gauss(seed, k, n, q, S_dev, dtype == RBFGS_F32 ? DT_F32 : DT_F64, n, (hipStream_t)hip_stream);
  return e == hipSuccess ? RBFGS_OK : RBFGS_E_DEVICE;
}

rbfgs_status rbfgs_sketch_coord(uint64_t seed, int64_t k, int64_t n, int32_t q, int32_t* idx_dev, void* hip_stream) {
  if (!idx_dev || n < 1 || q < 1 || q > n || k < 0 || n > (1ll << 20)) return RBFGS_E_INVALID_ARG;
  hipError_t e = sketch_coord(seed, k, n, q, idx_dev, (hipStream_t)hip_stream);
  return e == hipSuccess ? RBFGS_OK : RBFGS_E_DEVICE;
}

}  // extern "C"
