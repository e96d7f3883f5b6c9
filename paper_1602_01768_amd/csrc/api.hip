// C ABI of the RBFGS library: context management and the per-iteration
// orchestration of the kernels.  See include/rbfgs.h for the contract.
//
// Three HIP streams ("lanes") per context.  Everything of iteration k that depends
// only on the sketch is computed ahead of the X- (or L-) dependent part on the main
// lane, into one of three slots: the side lane forms S, A S and G = S^T A S (fixed
// method) or S~^T S~ (adaptive) up to two iterations ahead, the inverse lane the
// Cholesky-based inverse and U = S G^-1 one iteration ahead, so the long
// single-workgroup factorization of iteration k+1 overlaps the products of k+2
// and the main lane's work on k.  Events order the lanes.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/rbfgs.h"
#include "common.hpp"
#include "importance.hpp"
#include "kernels.hpp"
#include "pool.hpp"

using namespace rb;

// Device array behind rbfgs_ridge_hessian_noalloc.  Host code never passes `scratch` itself
// (on the host it names a stand-in, not device memory): each device's address of its copy is
// looked up once with hipGetSymbolAddress, with that device current, and kept in scratch_dev.
static __device__ __align__(256) unsigned char scratch[RBFGS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[SCRATCH_MAX_DEVICES] = {};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// This device's copy of `scratch` (the current device's).
hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

constexpr int POWER_STEPS = 100;  // power-method steps of the Newton-Schulz starting point
constexpr int SUPER_TILES = 4;    // super-tile edge of the n x n update order (4 x 4 tiles share panels in L2)

namespace {

constexpr int PROBES = 64;  // Gaussian probe vectors of the AdaRBFGS stopping test (relative std <= 18%)

struct Lane {  // one stream with its own split-K, reduction and Cholesky workspaces
  hipStream_t s = nullptr;
  void* partial = nullptr;
  size_t partial_bytes = 0;
  double* red = nullptr;
  size_t red_count = 0;
  double* cwork = nullptr;
  __bf16* bsplit = nullptr;  // bf16 planes of the panel of a streamed n x n product (mixed)
};

struct Slot {  // sketch-dependent quantities of one iteration
  void* Sk = nullptr;        // Gaussian sketch (S or S~), bf16 in mixed mode, FP64 otherwise
  int32_t* C = nullptr;      // coordinate indices
  void* Y = nullptr;         // fixed: A S
  double* G = nullptr;       // fixed: S^T A S;  adaptive: S~^T S~;  PSB, Kaczmarz: Y^T Y
  double* G2 = nullptr;      // PSB: S^T Y
  double* Ginv = nullptr;    // fixed: G^-1
  float* Ginv32 = nullptr;   // fixed, q-sized products in bf16: G^-1 rounded to FP32
  double* Z = nullptr;       // inverse Cholesky factor of G (fixed) or of S~^T S~ (adaptive)
  void* U = nullptr;         // fixed: U = S G^-1 (mixed: FP32 n x q; FP64: panels [U | W' | U])
  __bf16* planes = nullptr;  // mixed fixed: bf16 planes (hi, lo or hi, mid, lo) of [U | W' | U], tile-major
  double* ht = nullptr;      // partition sampling: 1/p_i of the drawn block (Horvitz-Thompson)
  hipEvent_t y_ready = nullptr;   // side lane: sketch and Y = A S written (fixed sketch)
  hipEvent_t g_ready = nullptr;   // side lane: G (or S~^T S~) written
  hipEvent_t ready = nullptr;     // inverse lane: slot complete
  hipEvent_t released = nullptr;  // main lane: iteration that used the slot complete
  bool released_valid = false;
};

}  // namespace

struct rbfgs_ctx {
  rbfgs_params p{};
  int64_t n = 0, np = 0, qp = 0;
  int q = 0;
  bool mixed = false, ada = false, coord = false;
  // other instances of the family: PSB (Alg. 3, W = I), AIP and Kaczmarz (Alg. 1 with
  // W = A^-1 or W = I; "row variants", nonsymmetric iterates); coordinate sketches of
  // these are used as dense 0/1 matrices (dcoord), `coord` marks the gather paths of
  // fixed RBFGS and AdaRBFGS only
  bool psb = false, rowv = false, kacz = false, dcoord = false;
  // mixed fixed RBFGS with a Gaussian sketch and streamed products: X is held on its lower
  // 128 x 128 tiles (the update writes no mirrored tiles; X Y reads the tiles right of the
  // diagonal transposed).  x_lower: the upper tiles are stale, and are copied from the lower
  // ones before anything reads X whole (residual, rbfgs_get_x, PCG)
  bool lowx = false, x_lower = false;
  // mixed symmetric update (fixed RBFGS, PSB) with q > n / 8: U and W' in three bf16 pieces (a
  // CPU emulation of the step on the ridge Hessian, n = 1024, q = 256, 40 steps: 1.16e-4 against
  // the oracle with two pieces, 6.9e-5 with three; n = 2048, q = 256: 2.4e-5 with two)
  bool upd3 = false;
  // partition sampling (fixed RBFGS, AdaRBFGS): the coordinate block C_i = [iq, (i+1)q) is
  // drawn with p_i proportional to Tr(S_i^T A S_i) (eq. ihsih0); tw holds the per-coordinate
  // weights, A_jj for the fixed method and (L^T A L)_jj for AdaRBFGS (updated every step)
  bool part = false;
  double* tw = nullptr;
  // importance sampling for Kaczmarz (eq. discoptprob with W = I and X_k in place of A^-1):
  // block i of the same partition with p_i proportional to ||X_k I_{:C_i} I_{C_i:} A||_F =
  // <(Z Z^T)_{C_i C_i}, (A A^T)_{C_i C_i}>^(1/2), recomputed from Z = X_k^T at every step;
  // BA holds the r blocks (A A^T)_{C_i C_i}, Pz q rows as a panel (to form BA), ipart the
  // partial sums of the batched weight kernel
  bool imp = false;
  double *BA = nullptr, *ipart = nullptr;
  int64_t ipart_cap = 0;
  void* Pz = nullptr;
  // comparison methods of Sec. 10 (FP64 only): Newton-Schulz and MR, n^3 products per step
  bool ns = false, mr = false;
  double *T2 = nullptr, *P2 = nullptr, *Q2 = nullptr;  // n x n FP64 work matrices
  double* scal = nullptr;                              // device scalars (sigma, ratios)
  int mdt = DT_F64;  // element type of A, X/L and the n x q panels
  int device = 0;
  int64_t k = 0;
  std::string err;
  static constexpr int NSLOT = 3;
  Lane main, side, inv;
  Slot slot[NSLOT];
  hipEvent_t ev_begin = nullptr;
  hipEvent_t ev_xy = nullptr;  // main lane: X Y of the current iteration enqueued before it
  hipEvent_t ev_g = nullptr, ev_chol = nullptr;  // adaptive: G formed (main), its inverse done (inverse lane)
  // main-lane buffers
  void* A = nullptr;
  void* X = nullptr;        // X (fixed, PSB), L (adaptive), X^T (AIP, Kaczmarz: the products read it k-contiguous)
  int32_t* pos = nullptr;   // inverse map of the coordinate set (-1 elsewhere)
  void* Sa = nullptr;       // adaptive: S = L S~
  void* Y = nullptr;        // adaptive: Y = A S
  void* V = nullptr;        // V = X Y (fixed) or T^T = L^T Y (adaptive)
  void* W = nullptr;        // fixed: W' (mixed) / copy of V (coordinates); adaptive: Q^T
  __bf16* planes = nullptr; // adaptive mixed: bf16 planes of S and Q^T
  void* R = nullptr;        // fixed coordinate: R = G^-1 W'^T (qp x np)
  double *G = nullptr, *H = nullptr, *Ginv = nullptr, *Z = nullptr, *GH = nullptr, *Mq = nullptr;
  float* H32 = nullptr;  // H in FP32 when H and U H run in bf16
  // mixed fixed Gaussian with qp a multiple of 128: G = S^T Y and U = S G^-1 as split-bf16
  // products (FP32 accumulation, FP64 sums of the split-K partials); H = Y^T V and U H too
  // when q <= n/8 (for larger q/n on ill-conditioned A their FP32 accumulation measurably
  // raised the error against the oracle, so they stay FP64 there)
  bool bf16q = false, bf16h = false;
  // est[0] the last step's estimate, est[1] scratch of the exact residual, est[2] the
  // window sum of the estimates, est[4] the probe estimate of AdaRBFGS (est[6] its scratch)
  double* est = nullptr;
  double* prb = nullptr;  // adaptive: Gaussian probes and two work panels, FP64 np x PROBES each
  int* status = nullptr;
  // n x n scratch allocated once: AdaRBFGS forms A L (exact residual) or L L^T (rbfgs_get_x)
  // in FP64 there; the row variants transpose their stored X^T into it (rbfgs_get_x)
  void* sq = nullptr;
  // staging for host transfers of n x n matrices, taken in row chunks
  void* stage = nullptr;
  size_t stage_bytes = 0;
  int2* tiles = nullptr;    // tile order of the n x n update (super-tiles, see make_tile_order)
  int64_t ntiles = 0;
  std::vector<void*> allocs;
  int64_t bytes = 0;  // device bytes the context holds (allocate() accounts them)
  rb::DevicePool* pool = nullptr;  // serving: buffers from the server's arena instead of hipMalloc
  bool own_lanes = true;           // false: every lane on the caller's stream (serving)
  // serving: a window of check_every steps is captured once into a HIP graph and replayed;
  // the sketch's iteration is then read from the device counter kdev (plus the step's offset
  // in the window, while kcap0 >= 0 during the capture), which the graph advances at its end
  int64_t* kdev = nullptr;
  // the side lanes' work is enqueued up to iteration prod_hi (products) and inv_hi (inverse):
  // enqueue_steps ends by issuing the next window's first products and inverse, so that a
  // window does not start with the side lanes idle (reset by rbfgs_set_state)
  int64_t prod_hi = -1, inv_hi = -1;
  int64_t kcap0 = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool dry = false;   // allocate() only sums sizes (rbfgs_footprint)
  // per-phase timing with HIP events on the lanes' streams (rbfgs_profile)
  struct ProfRec {
    std::string name;
    hipEvent_t a, b;
  };
  int prof = 0;  // 0 off, 1 every phase, 2 the n x n products only
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

// Order lane s after event e.  A serving context runs every lane on one stream, where stream
// order already holds -- and a wait on an event recorded before a graph capture began would
// break the capture -- so it skips the wait.
#define LANE_WAIT(s, e)                                         \
  do {                                                          \
    if (ctx->own_lanes) HIPCHK(hipStreamWaitEvent((s), (e), 0)); \
  } while (0)

// Zeroed device allocation owned by the context.  In a dry run (footprint) only the
// size is accounted and a placeholder is returned.
void* dalloc(rbfgs_ctx* ctx, size_t bytes) {
  const size_t b = bytes ? bytes : 16;
  ctx->bytes += (int64_t)((b + 255) / 256 * 256);
  if (ctx->dry) return (void*)(uintptr_t)256;
  void* p = nullptr;
  if (ctx->pool) {
    p = ctx->pool->alloc(b);
    if (!p) {
      ctx->err = "the server's device memory pool has no free run of this size";
      throw Fail{RBFGS_E_OOM};
    }
  } else {
    HIPCHK(hipMalloc(&p, b));
  }
  ctx->allocs.push_back(p);
  HIPCHK(hipMemsetAsync(p, 0, b, ctx->main.s));
  return p;
}

// A roctx range for the scope (host side: it spans the launches made inside it).
struct RocRange {
  explicit RocRange(const char* n) { roctxRangePushA(n); }
  ~RocRange() { roctxRangePop(); }
  RocRange(const RocRange&) = delete;
  RocRange& operator=(const RocRange&) = delete;
};

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

// Scope that brackets the kernels of one phase with events on one lane.  `product`
// marks the n x n products (timed at profile level 2 as well); for those, mark()
// gives an event that the split-K GEMM records between its product kernel and the
// reduction, which is then reported as the separate phase "<name>.reduce".  Every phase
// is also a roctx range around its launches (recorded by rocprofv3 --marker-trace).
struct Phase {
  rbfgs_ctx* ctx;
  hipStream_t s;
  const char* name;
  hipEvent_t a = nullptr, mid = nullptr;
  RocRange range;
  Phase(rbfgs_ctx* c, const Lane& L, const char* n, bool product = false) : ctx(c), s(L.s), name(n), range(n) {
    if (ctx->prof == 1 || (ctx->prof == 2 && product)) {
      a = prof_event(ctx);
      HIPCHK(hipEventRecord(a, s));
    }
  }
  hipEvent_t mark() {
    if (a && !mid) mid = prof_event(ctx);
    return mid;
  }
  ~Phase() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (!ctx->ev_pool.empty()) {
      b = ctx->ev_pool.back();
      ctx->ev_pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
      return;
    }
    if (hipEventRecord(b, s) != hipSuccess) return;
    if (mid) {
      ctx->prof_pending.push_back({name, a, mid});
      ctx->prof_pending.push_back({std::string(name) + ".reduce", mid, b});
    } else {
      ctx->prof_pending.push_back({name, a, b});
    }
  }
};

void prof_flush(rbfgs_ctx* ctx) {
  if (ctx->prof_pending.empty()) return;
  HIPCHK(hipStreamSynchronize(ctx->main.s));
  HIPCHK(hipStreamSynchronize(ctx->side.s));
  HIPCHK(hipStreamSynchronize(ctx->inv.s));
  std::vector<hipEvent_t> used;
  for (auto& r : ctx->prof_pending) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    auto& acc = ctx->prof_acc[r.name];
    acc.first += ms;
    acc.second += 1;
    used.push_back(r.a);
    used.push_back(r.b);
  }
  std::sort(used.begin(), used.end());
  used.erase(std::unique(used.begin(), used.end()), used.end());
  for (hipEvent_t e : used) ctx->ev_pool.push_back(e);
  ctx->prof_pending.clear();
}

// Split-K factor: enough workgroups to fill the chip (>= 1024) with K chunks of at
// least min_chunk; at most max_split partial buffers.
// split-K grows until tiles x splits reaches this many workgroups.  At n = 16384, q = 256
// (128 row tiles): 1024 (split 8) 565 iterations/s, 512 (split 4) 558, 256 (split 2) 573, the
// last by running A S longer, beside the update; 1024 is kept
constexpr int64_t SPLIT_TARGET = 1024;
int pick_split(int64_t tiles, int64_t K, int kmul, int max_split = 8, int64_t min_chunk = 256) {
  int s = 1;
  while (s < max_split && tiles * s < SPLIT_TARGET && K % ((int64_t)kmul * s * 2) == 0 && K / (s * 2) >= min_chunk)
    s *= 2;
  return s;
}

int64_t f64_tile(int64_t x) { return x % 128 == 0 ? 128 : 32; }
int64_t bf_bn(int64_t N) { return N % 256 == 0 ? 256 : (N % 128 == 0 ? 128 : (N % 64 == 0 ? 64 : 32)); }

// FP64-MFMA product on one lane; column-store products get a split-K.
void f64_gemm(rbfgs_ctx* ctx, const Lane& L, GemmArgs g) {
  if (g.epi == EPI_COLSTORE) {
    const bool small_out = g.M * g.N <= (int64_t)1024 * 1024;  // q x q products: split deep
    if (small_out) {
      const int64_t t = (g.M % 64 == 0 && g.N % 64 == 0) ? 64 : 32;
      g.splitk = pick_split((g.M / t) * (g.N / t), g.K, 16, 32, 256);
    } else {
      g.splitk = pick_split((g.M / f64_tile(g.M)) * (g.N / f64_tile(g.N)), g.K, 16);
    }
    const size_t need = (size_t)g.splitk * g.M * g.N * sizeof(double);
    if (g.splitk > 1 && need > L.partial_bytes) g.splitk = 1;
  }
  HIPCHK(gemm_f64(g, L.partial, L.s));
}

// Split-K factor of a tall-skinny bf16 product on lane L.
int bf_split(rbfgs_ctx* ctx, const Lane& L, const MixedGemm& mg, int max_split = 8, int64_t min_chunk = 256) {
  const GemmArgs& g = mg.g;
  const int64_t tiles = (g.M / 128) * (g.N / (g.bn ? g.bn : bf_bn(g.N)));
  const int s = pick_split(tiles, g.K, 32, max_split, min_chunk);
  return (size_t)s * g.M * g.N * sizeof(float) > L.partial_bytes ? 1 : s;
}

// bf16-MFMA product on one lane (tall-skinny products get a split-K).
void bf_gemm(rbfgs_ctx* ctx, const Lane& L, MixedGemm mg, int max_split = 8, int64_t min_chunk = 256) {
  GemmArgs& g = mg.g;
  if (g.epi == EPI_COLSTORE) g.splitk = bf_split(ctx, L, mg, max_split, min_chunk);
  HIPCHK(gemm_bf16(mg, L.partial, L.s));
}

// q x q Gram C = P1^T P2 of two n x q column-major panels as a split-bf16 product:
// P1 in p1_pieces (1 for the exact bf16 sketch), P2 FP32 in 3 pieces, all piece pairs of
// weight >= 2^-16; FP32 accumulation over 64-wide k chunks, chunks summed in double.
void gram_bf16(rbfgs_ctx* ctx, const Lane& L, const void* P1, bool p1_bf16, const float* P2, void* out, int out_dt) {
  MixedGemm mg;
  GemmArgs& g = mg.g;
  g.M = ctx->qp; g.N = ctx->qp; g.K = ctx->np;
  g.A = P1; g.lda = ctx->np;
  g.B = P2; g.ldb = ctx->np;
  g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->qp; g.c_dt = out_dt; g.c2 = 1.0;
  g.bn = 128;
  mg.a_kind = p1_bf16 ? OK_BF16_KC : OK_F32_KC; mg.b_kind = OK_F32_KC;
  mg.na = p1_bf16 ? 1 : 3; mg.nb = 3; mg.pmax = 2;
  bf_gemm(ctx, L, mg, 64, 256);
}

// out = M * P for an n x n matrix M (A, X or L) and an n x q panel P, per precision.
// transpose: Aop = M^T (T^T = L^T Y).  In mixed mode (na, nb, pmax) choose the bf16
// pieces of each operand and the passes kept (all piece pairs with i + j <= pmax).
// est_S (mixed mode): the reduction of the product also accumulates per-workgroup sums
// of (est_S - out)^2 into L.red (see reduce_blocks_f32).
// lower: M is symmetric and current on its lower 128 x 128 tiles only (streamed product).
void nn_times_panel(rbfgs_ctx* ctx, const Lane& L, const void* M, bool transpose, const void* P, int p_dt, void* out,
                    int na = 2, int nb = 2, int pmax = 1, hipEvent_t mark = nullptr, const __bf16* est_S = nullptr,
                    bool lower = false) {
  if (ctx->mixed) {
    MixedGemm mg;
    GemmArgs& g = mg.g;
    g.M = ctx->np; g.N = ctx->qp; g.K = ctx->np;
    g.A = M; g.lda = ctx->np;
    g.B = P; g.ldb = ctx->np;
    g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->np; g.c_dt = DT_F32; g.c2 = 1.0; g.mark = mark;
    if (est_S) {
      g.est_S = est_S;
      g.est_red = L.red;
    }
    mg.a_kind = transpose ? OK_F32_MC : OK_F32_KC;
    mg.b_kind = p_dt == DT_BF16 ? OK_BF16_KC : OK_F32_KC;
    mg.na = na; mg.nb = p_dt == DT_BF16 ? 1 : nb; mg.pmax = pmax;
    // streamed product: an FP32 panel is split into bf16 planes once, here, instead of in
    // every row tile of the product (a bf16 panel is copied), the planes tile-major so that
    // each 32-deep k tile of the panel is one contiguous block
    if (L.bsplit) {
      MixedGemm sm = mg;
      if (lower) sm.a_kind = OK_F32_SYM;
      sm.b_kind = OK_BF16_KC;
      sm.g.B = L.bsplit; sm.g.ldb = ctx->qp; sm.g.b_plane = ctx->np * ctx->qp; sm.g.b_tiled = true;
      sm.g.splitk = bf_split(ctx, L, sm);
      if (tall_stream_supported(sm)) {
        HIPCHK(split_planes(P, ctx->np, ctx->qp, ctx->np, sm.nb, L.bsplit, L.s));
        mg = sm;
      }
    }
    if (lower && mg.a_kind != OK_F32_SYM) {  // (lowx is set only where the streamed product applies)
      ctx->err = "an operand held on its lower tiles needs the streamed product";
      throw Fail{RBFGS_E_DEVICE};
    }
    bf_gemm(ctx, L, mg);
  } else {
    GemmArgs g;
    g.M = ctx->np; g.N = ctx->qp; g.K = ctx->np;
    g.A = M; g.lda = ctx->np; g.a_dt = DT_F64; g.a_kc = !transpose;
    g.B = P; g.ldb = ctx->np; g.b_dt = p_dt; g.b_kc = true;
    g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->np; g.c_dt = DT_F64; g.c2 = 1.0; g.mark = mark;
    f64_gemm(ctx, L, g);
  }
}

// q x q Gram C = P1^T P2 of two n x q column-major panels, FP64 accumulation.
void gram(rbfgs_ctx* ctx, const Lane& L, const void* P1, int dt1, const void* P2, int dt2, double* out) {
  GemmArgs g;
  g.M = ctx->qp; g.N = ctx->qp; g.K = ctx->np;
  g.A = P1; g.lda = ctx->np; g.a_dt = dt1; g.a_kc = true;
  g.B = P2; g.ldb = ctx->np; g.b_dt = dt2; g.b_kc = true;
  g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->qp; g.c_dt = DT_F64; g.c2 = 1.0;
  f64_gemm(ctx, L, g);
}

// out(n x q) = c2 * P(n x q, col-major) * M(q x q, row-major) [+ c0*B0 + c1*B1]
void panel_times_small(rbfgs_ctx* ctx, const Lane& L, const void* P, int p_dt, const double* M, void* out, int out_dt,
                       double c2, const void* B0 = nullptr, int b0_dt = DT_F64, double c0 = 0,
                       const void* B1 = nullptr, int b1_dt = DT_F64, double c1 = 0) {
  GemmArgs g;
  g.M = ctx->np; g.N = ctx->qp; g.K = ctx->qp;
  g.A = P; g.lda = ctx->np; g.a_dt = p_dt; g.a_kc = false;
  g.B = M; g.ldb = ctx->qp; g.b_dt = DT_F64; g.b_kc = false;
  g.epi = EPI_COLSTORE; g.C = out; g.ldc = ctx->np; g.c_dt = out_dt; g.c2 = c2;
  g.B0 = B0; g.b0_dt = b0_dt; g.c0 = c0; g.B1 = B1; g.b1_dt = b1_dt; g.c1 = c1; g.ld01 = ctx->np;
  f64_gemm(ctx, L, g);
}

// out(q x q, row-major) = Aop * Bop with row-major q x q inputs (transposes by flag).
void small_small(rbfgs_ctx* ctx, const Lane& L, const double* A, bool at, const double* B, double* out) {
  GemmArgs g;
  g.M = ctx->qp; g.N = ctx->qp; g.K = ctx->qp;
  g.A = A; g.lda = ctx->qp; g.a_dt = DT_F64; g.a_kc = !at;
  g.B = B; g.ldb = ctx->qp; g.b_dt = DT_F64; g.b_kc = false;
  g.epi = EPI_ROWSTORE; g.C = out; g.ldc = ctx->qp; g.c_dt = DT_F64; g.c2 = 1.0;
  f64_gemm(ctx, L, g);
}

int sk_dt(const rbfgs_ctx* ctx) { return ctx->mixed ? DT_BF16 : DT_F64; }

// (M M^T)_{CC} for the q rows C = [bq, (b+1)q) of the row-major np x np matrix M (A, or
// Z = X^T for the row variants): the rows, contiguous in memory, are the first q columns of
// the column-major panel Pz (its other columns are zero), and out (qp x qp) = Pz^T Pz.
void row_block_gram(rbfgs_ctx* ctx, const Lane& L, const void* M, int64_t b, double* out) {
  const size_t es = dt_size(ctx->mdt);
  HIPCHK(hipMemcpyAsync(ctx->Pz, (const char*)M + (size_t)b * ctx->q * ctx->np * es, (size_t)ctx->q * ctx->np * es,
                        hipMemcpyDeviceToDevice, L.s));
  gram(ctx, L, ctx->Pz, ctx->mdt, ctx->Pz, ctx->mdt, out);
}

// Kaczmarz with importance sampling: the weights ||X_k I_{:C_i} I_{C_i:} A||_F of every block
// from the current Z = X_k^T (one batched launch over all blocks), then the draw of
// iteration k into the slot (main lane).
void importance_draw(rbfgs_ctx* ctx, Slot& S, int64_t k) {
  const Lane& L = ctx->main;
  Phase ph(ctx, L, "importance");
  HIPCHK(block_gram_weights(ctx->X, ctx->mdt, ctx->np, ctx->n, (int)ctx->q, ctx->BA, ctx->qp, ctx->ipart,
                            ctx->ipart_cap, ctx->tw, L.s));
  HIPCHK(sample_partition(ctx->tw, ctx->n, ctx->q, ctx->p.seed, k, S.C, S.ht, ctx->status, L.s));
}

// Row-tile height of the tile-major bf16 panel planes of the n x n update: its tile edge (the
// symmetric update of the fixed method and PSB, or the full-square one of AdaRBFGS and the row
// variants).
int64_t upd_panel_tile(const rbfgs_ctx* ctx) {
  return ctx->ada || ctx->rowv ? bf16_square_tile(ctx->np, ctx->qp, EPI_ADDROW)
                               : bf16_square_tile(ctx->np, 2 * ctx->qp, EPI_SYMUPD);
}

// ---------------------------------------------------------------- side lanes
// Sketch-dependent products of iteration k into slot S (side lane): the sketch, and
// for the fixed method Y = A S (or the gathered columns) and G = S^T Y; for the
// adaptive Gaussian method S~^T S~.
void side_products(rbfgs_ctx* ctx, int64_t k, Slot& S) {
  const Lane& L = ctx->side;
  const int64_t np = ctx->np, qp = ctx->qp;
  const int mdt = ctx->mdt;
  {
    Phase ph(ctx, L, "sketch");
    if (ctx->imp) {
      // drawn on the main lane (the weights depend on X_k)
    } else if (ctx->part) {
      // fixed: static weights, drawn ahead; AdaRBFGS draws on the main lane (its weights
      // depend on the previous step)
      if (!ctx->ada) HIPCHK(sample_partition(ctx->tw, ctx->n, ctx->q, ctx->p.seed, k, S.C, S.ht, ctx->status, L.s));
    } else if (ctx->coord || ctx->dcoord) HIPCHK(sketch_coord(ctx->p.seed, k, ctx->n, ctx->q, S.C, L.s));
    else if (ctx->kcap0 >= 0)
      HIPCHK(sketch_gauss(ctx->p.seed, k - ctx->kcap0, ctx->n, ctx->q, S.Sk, sk_dt(ctx), np, L.s, ctx->kdev));
    else HIPCHK(sketch_gauss(ctx->p.seed, k, ctx->n, ctx->q, S.Sk, sk_dt(ctx), np, L.s));
    if (ctx->dcoord) HIPCHK(coord_dense(S.C, ctx->q, S.Sk, sk_dt(ctx), np, qp, L.s));
  }
  if (ctx->ada) {
    if (!ctx->coord) {
      Phase ph(ctx, L, "sketch_gram");
      gram(ctx, L, S.Sk, sk_dt(ctx), S.Sk, sk_dt(ctx), S.G);
    }
  } else if (ctx->coord) {
    Phase ph(ctx, L, "gather");
    HIPCHK(gather_cols_sym(ctx->A, mdt, np, S.C, ctx->q, np, S.Y, mdt, np, S.G, qp, L.s));
    HIPCHK(hipEventRecord(S.y_ready, L.s));
  } else {
    {
      // Y = A S (Kaczmarz: P = A^T S)
      Phase ph(ctx, L, "AS", true);
      nn_times_panel(ctx, L, ctx->A, ctx->kacz, S.Sk, sk_dt(ctx), S.Y, 3, 1, 2, ph.mark());  // exact
    }
    HIPCHK(hipEventRecord(S.y_ready, L.s));
    Phase ph(ctx, L, "gram_G");
    if (ctx->bf16q) gram_bf16(ctx, L, S.Sk, true, (const float*)S.Y, S.G, DT_F64);
    else if (ctx->psb || ctx->kacz) gram(ctx, L, S.Y, mdt, S.Y, mdt, S.G);  // S^T A^2 S, S^T A A^T S
    else gram(ctx, L, S.Sk, sk_dt(ctx), S.Y, mdt, S.G);
    if (ctx->psb) gram(ctx, L, S.Sk, sk_dt(ctx), S.Y, mdt, S.G2);
  }
  HIPCHK(hipEventRecord(S.g_ready, L.s));
}

// Inverse part of iteration k into slot S (inverse lane), after side_products: the
// Cholesky-based inverse of G (fixed) or the factor of S~^T S~ (adaptive Gaussian),
// and U = S G^-1 packed for the update (fixed Gaussian).
void side_inverse(rbfgs_ctx* ctx, Slot& S) {
  const Lane& L = ctx->inv;
  const int64_t np = ctx->np, qp = ctx->qp;
  if (ctx->ada) {
    if (!ctx->coord) {  // factor of S~^T S~ for C = L_M^-1
      Phase ph(ctx, L, "sketch_chol");
      HIPCHK(chol_inv(S.G, qp, ctx->q, S.Z, nullptr, qp, L.cwork, ctx->status, L.s));
    }
    return;
  }
  { Phase ph(ctx, L, "chol_inv"); HIPCHK(chol_inv(S.G, qp, ctx->q, S.Z, S.Ginv, qp, L.cwork, ctx->status, L.s)); }
  if (ctx->coord) return;
  Phase ph(ctx, L, "panel_U");
  if (ctx->mixed) {
    float* U = (float*)S.U;
    if (ctx->bf16q) {  // U = S G^-1: S exact bf16 (m-contiguous), G^-1 rounded to FP32 in 3 pieces
      HIPCHK(copy_convert(S.Ginv, DT_F64, qp, S.Ginv32, DT_F32, qp, qp, qp, L.s));
      MixedGemm mg;
      GemmArgs& g = mg.g;
      g.M = np; g.N = qp; g.K = qp;
      g.A = S.Sk; g.lda = np;
      g.B = S.Ginv32; g.ldb = qp;  // Bop(k, j) = G^-1[j][k] = G^-1[k][j]
      g.epi = EPI_COLSTORE; g.C = U; g.ldc = np; g.c_dt = DT_F32; g.c2 = 1.0; g.bn = 128;
      mg.a_kind = OK_BF16_MC; mg.b_kind = OK_F32_KC; mg.na = 1; mg.nb = 3; mg.pmax = 2;
      bf_gemm(ctx, L, mg, 1);  // k = q is short: no split
    } else if (ctx->psb || ctx->kacz) {
      panel_times_small(ctx, L, S.Y, DT_F32, S.Ginv, U, DT_F32, 1.0);  // U = Y G^-1
    } else {
      panel_times_small(ctx, L, S.Sk, DT_BF16, S.Ginv, U, DT_F32, 1.0);
    }
    // [U W' U] for the symmetric update, or U for the row variants' update; pieces hi, lo or
    // hi, mid, lo in planes 0, 1(, 2)
    const int64_t ldp = 3 * qp, plane = np * ldp, tile = upd_panel_tile(ctx);
    __bf16* lo = S.planes + (ctx->upd3 ? 2 : 1) * plane;
    __bf16* mid = ctx->upd3 ? S.planes + plane : nullptr;
    HIPCHK(pack_split2(U, np, np, qp, S.planes, lo, ldp, 0, L.s, tile, mid));
    HIPCHK(pack_split2(U, np, np, qp, S.planes, lo, ldp, 2 * qp, L.s, tile, mid));
  } else {
    double* U = (double*)S.U;
    if (ctx->psb || ctx->kacz) panel_times_small(ctx, L, S.Y, DT_F64, S.Ginv, U, DT_F64, 1.0);  // U = Y G^-1
    else panel_times_small(ctx, L, S.Sk, DT_F64, S.Ginv, U, DT_F64, 1.0);
    HIPCHK(hipMemcpyAsync(U + 2 * np * qp, U, (size_t)np * qp * sizeof(double), hipMemcpyDeviceToDevice, L.s));
  }
}

// ---------------------------------------------------------------- main lane
// X-dependent part of one fixed-sketch RBFGS iteration, eq. (qunac) as the
// symmetric rank-2q update X+ = X - (U W'^T + W' U^T), U = S G^-1,
// W' = V - S/2 - U H/2, V = X Y, H = Y^T V (Y = A S and G = S^T Y from the slot).
// `after_xy` is called once V = X Y is enqueued, `ahead` once, at the point where the
// side lanes' remaining work for later iterations is to be released (before the update
// of X, or earlier on the paths that have no separate update).
template <class F, class G>
void main_fixed(rbfgs_ctx* ctx, Slot& S, G&& after_xy, F&& ahead) {
  const Lane& L = ctx->main;
  bool fired = false;
  auto release = [&]() {
    if (!fired) ahead();
    fired = true;
  };
  const int64_t np = ctx->np, qp = ctx->qp;
  const int mdt = ctx->mdt;
  // mixed Gaussian: the estimator's sum of squares comes out of the product's reduction
  GemmArgs shape;
  shape.M = np; shape.N = qp;
  const bool fused_est = ctx->mixed && !ctx->coord && (size_t)reduce_blocks_f32(shape) <= L.red_count;
  {
    Phase ph(ctx, L, "XY", true);
    nn_times_panel(ctx, L, ctx->X, false, S.Y, mdt, ctx->V, 2, 2, 1, ph.mark(),
                   fused_est ? (const __bf16*)S.Sk : nullptr, ctx->lowx);
  }
  after_xy();
  {
    Phase ph(ctx, L, "gram_H");
    if (ctx->bf16h) gram_bf16(ctx, L, S.Y, false, (const float*)ctx->V, ctx->H32, DT_F32);
    else gram(ctx, L, S.Y, mdt, ctx->V, mdt, ctx->H);
  }
  // partition: the Horvitz-Thompson factor 1/p_i of the drawn block, read on the device
  const double scale = ctx->part ? 1.0 : (ctx->coord || ctx->dcoord) ? (double)ctx->n / ctx->q : 1.0 / ctx->q;
  {
    Phase ph(ctx, L, "estimator");
    if (fused_est)
      HIPCHK(reduce_sum_scaled(L.red, reduce_blocks_f32(shape), ctx->est, scale, ctx->status, L.s));
    else
      HIPCHK(estimator(ctx->coord ? nullptr : S.Sk, sk_dt(ctx), ctx->coord ? S.C : nullptr, ctx->V, mdt, np, ctx->n,
                       ctx->q, scale, L.red, ctx->est, ctx->status, L.s, ctx->part ? S.ht : nullptr));
  }
  LANE_WAIT(L.s, S.ready);  // G^-1 and U of this slot
  // PSB: H' = Y^T V - S^T Y (= R^T Y with R = V - S), and W' = V - S - U H'/2
  const double cs = ctx->psb ? -1.0 : -0.5;
  if (ctx->psb) HIPCHK(panel_axpby(ctx->H, DT_F64, 1.0, S.G2, DT_F64, -1.0, ctx->H, DT_F64, qp, qp, qp, L.s));
  if (ctx->coord) {
    // U = E_C G^-1 is not formed: W' = V - E_C/2 - E_C (G^-1 H)/2 and R = G^-1 W'^T;
    // the update touches only rows and columns C.
    release();
    Phase ph(ctx, L, "coord_update");
    small_small(ctx, L, S.Ginv, false, ctx->H, ctx->GH);
    HIPCHK(hipMemcpyAsync(ctx->W, ctx->V, (size_t)np * qp * dt_size(mdt), hipMemcpyDeviceToDevice, L.s));
    HIPCHK(coord_wprime_fix(ctx->W, mdt, np, S.C, ctx->q, ctx->GH, qp, L.s));
    GemmArgs g;
    g.M = qp; g.N = np; g.K = qp;
    g.A = S.Ginv; g.lda = qp; g.a_dt = DT_F64; g.a_kc = true;
    g.B = ctx->W; g.ldb = np; g.b_dt = mdt; g.b_kc = false;
    g.epi = EPI_ROWSTORE; g.C = ctx->R; g.ldc = np; g.c_dt = mdt; g.c2 = 1.0;
    f64_gemm(ctx, L, g);
    HIPCHK(coord_sym_update(ctx->X, mdt, np, S.C, ctx->pos, ctx->q, np, ctx->R, mdt, np, L.s));
    return;
  }
  if (ctx->mixed) {
    float* W = (float*)ctx->W;
    const int64_t ldp = 3 * qp, plane = np * ldp;
    {
      Phase ph(ctx, L, "panels");
      if (ctx->bf16h) {  // W' = V - S/2 - (U H)/2, U in 3 pieces (m-contiguous), H in 3 pieces
        MixedGemm mg;
        GemmArgs& g = mg.g;
        g.M = np; g.N = qp; g.K = qp;
        g.A = S.U; g.lda = np;
        g.B = ctx->H32; g.ldb = qp;  // Bop(k, j) = H[k][j] (column-major H)
        g.epi = EPI_COLSTORE; g.C = W; g.ldc = np; g.c_dt = DT_F32; g.c2 = -0.5;
        g.B0 = ctx->V; g.c0 = 1.0; g.B1 = S.Sk; g.b1_dt = DT_BF16; g.c1 = -0.5; g.ld01 = np; g.bn = 128;
        mg.a_kind = OK_F32_MC; mg.b_kind = OK_F32_KC; mg.na = 3; mg.nb = 3; mg.pmax = 2;
        bf_gemm(ctx, L, mg, 1);  // k = q is short: no split
      } else {
        panel_times_small(ctx, L, S.U, DT_F32, ctx->H, W, DT_F32, -0.5, ctx->V, DT_F32, 1.0, S.Sk, DT_BF16, cs);
      }
      HIPCHK(pack_split2(W, np, np, qp, S.planes, S.planes + (ctx->upd3 ? 2 : 1) * plane, ldp, qp, L.s,
                         upd_panel_tile(ctx), ctx->upd3 ? S.planes + plane : nullptr));
    }
    release();
    Phase ph(ctx, L, "update", true);
    MixedGemm mg;
    GemmArgs& g = mg.g;
    g.M = np; g.N = np; g.K = 2 * qp;
    // the planes are tile-major: column qp of a row tile starts qp x tile entries into its block
    g.A = S.planes; g.lda = ldp; g.a_plane = plane;
    g.B = S.planes + qp * upd_panel_tile(ctx); g.ldb = ldp; g.b_plane = plane;
    g.epi = EPI_SYMUPD; g.C = ctx->X; g.ldc = np; g.c2 = -1.0;
    g.tiles = ctx->tiles; g.ntiles = ctx->ntiles; g.bn = bf16_square_tile(np, g.K, g.epi);  // (the order's tiles)
    g.lower_only = ctx->lowx;
    mg.a_kind = OK_BF16_KC; mg.b_kind = OK_BF16_KC; mg.na = 2; mg.nb = 2; mg.pmax = 1;
    if (ctx->upd3) {
      mg.na = 3; mg.nb = 3; mg.pmax = 2;
      g.upd_pieces = 3;
    }
    bf_gemm(ctx, L, mg);
    ctx->x_lower = ctx->lowx;
  } else {
    double* PQ = (double*)S.U;  // [U | W' | U], column-major, ld = np
    {
      Phase ph(ctx, L, "panels");
      panel_times_small(ctx, L, PQ, DT_F64, ctx->H, PQ + np * qp, DT_F64, -0.5, ctx->V, DT_F64, 1.0, S.Sk, DT_F64,
                        cs);
    }
    release();
    Phase ph(ctx, L, "update", true);
    GemmArgs g;
    g.M = np; g.N = np; g.K = 2 * qp;
    g.A = PQ; g.lda = np; g.a_dt = DT_F64; g.a_kc = false;
    g.B = PQ + np * qp; g.ldb = np; g.b_dt = DT_F64; g.b_kc = false;
    g.epi = EPI_SYMUPD; g.C = ctx->X; g.ldc = np; g.c_dt = DT_F64; g.c2 = -1.0;
    g.tiles = ctx->tiles; g.ntiles = ctx->ntiles;
    f64_gemm(ctx, L, g);
  }
}

// X-dependent part of one step of a row variant of Alg. 1 (AIP, eq. BFGSas: P = A S,
// U = S G^-1, G = S^T P; simultaneous randomized Kaczmarz, eq. badbroyadj: P = A^T S,
// U = P G^-1, G = P^T P; P, G and U from the slot):
//   C = X^T P,  R = S - C  (R^T = S^T (I - A X), the residual sketch),  X+ = X + U R^T
// on every tile of X (the iterates are not symmetric).  The context stores Z = X^T, so
// that C = Z P reads Z k-contiguous like X Y, and the update is Z+ = Z + R U^T.  The
// estimator is ||R||_F^2.
template <class F, class G>
void main_row(rbfgs_ctx* ctx, Slot& S, G&& after_xy, F&& ahead) {
  const Lane& L = ctx->main;
  const int64_t np = ctx->np, qp = ctx->qp;
  const int mdt = ctx->mdt;
  GemmArgs shape;
  shape.M = np; shape.N = qp;
  const bool fused_est = ctx->mixed && !ctx->imp && (size_t)reduce_blocks_f32(shape) <= L.red_count;
  {
    Phase ph(ctx, L, "XtP", true);
    nn_times_panel(ctx, L, ctx->X, false, S.Y, mdt, ctx->V, 2, 2, 1, ph.mark(),
                   fused_est ? (const __bf16*)S.Sk : nullptr);
  }
  after_xy();
  // importance sampling: the Horvitz-Thompson factor 1/p_i of the drawn block
  const double scale = ctx->imp ? 1.0 : ctx->dcoord ? (double)ctx->n / ctx->q : 1.0 / ctx->q;
  {
    Phase ph(ctx, L, "estimator");
    if (fused_est)
      HIPCHK(reduce_sum_scaled(L.red, reduce_blocks_f32(shape), ctx->est, scale, ctx->status, L.s));
    else
      HIPCHK(estimator(S.Sk, sk_dt(ctx), nullptr, ctx->V, mdt, np, ctx->n, ctx->q, scale, L.red, ctx->est,
                       ctx->status, L.s, ctx->imp ? S.ht : nullptr));
  }
  LANE_WAIT(L.s, S.ready);  // U of this slot
  ahead();
  {
    Phase ph(ctx, L, "panels");
    HIPCHK(panel_axpby(S.Sk, sk_dt(ctx), 1.0, ctx->V, mdt, -1.0, ctx->W, mdt, np, qp, np, L.s));  // R = S - C
    if (ctx->mixed)
      HIPCHK(pack_split2((const float*)ctx->W, np, np, qp, ctx->planes, ctx->planes + np * qp, qp, 0, L.s,
                         upd_panel_tile(ctx)));
  }
  Phase ph(ctx, L, "update", true);  // Z = X^T += R U^T
  if (ctx->mixed) {
    const int64_t ldp = 3 * qp;
    MixedGemm mg;
    GemmArgs& g = mg.g;
    g.M = np; g.N = np; g.K = qp;
    g.A = ctx->planes; g.lda = qp; g.a_plane = np * qp;
    g.B = S.planes; g.ldb = ldp; g.b_plane = np * ldp;
    g.epi = EPI_ADDROW; g.C = ctx->X; g.ldc = np; g.c2 = 1.0;
    g.tiles = ctx->tiles; g.ntiles = ctx->ntiles; g.bn = bf16_square_tile(np, g.K, g.epi);
    mg.a_kind = OK_BF16_KC; mg.b_kind = OK_BF16_KC; mg.na = 2; mg.nb = 2; mg.pmax = 1;
    bf_gemm(ctx, L, mg);
  } else {
    GemmArgs g;
    g.M = np; g.N = np; g.K = qp;
    g.A = ctx->W; g.lda = np; g.a_dt = DT_F64; g.a_kc = false;
    g.B = S.U; g.ldb = np; g.b_dt = DT_F64; g.b_kc = false;
    g.epi = EPI_ADDROW; g.C = ctx->X; g.ldc = np; g.c_dt = DT_F64; g.c2 = 1.0;
    g.tiles = ctx->tiles; g.ntiles = ctx->ntiles;
    f64_gemm(ctx, L, g);
  }
}

// L-dependent part of one AdaRBFGS iteration, eq. (Cholimprov) with R = L_G^-T,
// C = L_M^-1 (L_M^-1 from the slot):
//   S = L S~,  Y = A S,  G = S^T Y = L_G L_G^T,  T^T = L^T Y,
//   Q^T = S~ (L_M^-T L_G^-1) - T^T G^-1,  L+ = L + S Q.
void main_adaptive(rbfgs_ctx* ctx, Slot& S, int64_t k) {
  const Lane& L = ctx->main;
  const int64_t np = ctx->np, qp = ctx->qp;
  const int mdt = ctx->mdt;
  if (ctx->part) {  // block drawn by the weights (L_k^T A L_k)_jj of eq. ihsih0
    Phase ph(ctx, L, "sample");
    HIPCHK(sample_partition(ctx->tw, ctx->n, ctx->q, ctx->p.seed, k, S.C, S.ht, ctx->status, L.s));
  }
  if (ctx->coord) {
    Phase ph(ctx, L, "gather");
    HIPCHK(gather_cols_gen(ctx->X, mdt, np, S.C, ctx->q, np, ctx->Sa, mdt, np, L.s));
  } else {
    Phase ph(ctx, L, "LS", true);
    nn_times_panel(ctx, L, ctx->X, false, S.Sk, sk_dt(ctx), ctx->Sa, 3, 1, 2, ph.mark());  // S = L S~, exact products
  }
  {
    Phase ph(ctx, L, "AS", true);
    nn_times_panel(ctx, L, ctx->A, false, ctx->Sa, mdt, ctx->Y, 3, 2, 2, ph.mark());
  }
  { Phase ph(ctx, L, "gram_G"); gram(ctx, L, ctx->Sa, mdt, ctx->Y, mdt, ctx->G); }
  // the q x q inverse (a latency-bound chain of small kernels) runs on the inverse lane while
  // the main lane forms T^T = L^T Y, which does not need it
  HIPCHK(hipEventRecord(ctx->ev_g, L.s));
  LANE_WAIT(ctx->inv.s, ctx->ev_g);
  {
    Phase ph(ctx, ctx->inv, "chol_inv");
    HIPCHK(chol_inv(ctx->G, qp, ctx->q, ctx->Z, ctx->Ginv, qp, ctx->inv.cwork, ctx->status, ctx->inv.s));
  }
  HIPCHK(hipEventRecord(ctx->ev_chol, ctx->inv.s));
  {
    Phase ph(ctx, L, "LtY", true);
    nn_times_panel(ctx, L, ctx->X, true, ctx->Y, mdt, ctx->V, 2, 3, 2, ph.mark());  // T^T = L^T Y
  }
  LANE_WAIT(L.s, ctx->ev_chol);
  const double scale = ctx->part ? 1.0 : ctx->coord ? (double)ctx->n / ctx->q : 1.0 / ctx->q;
  {
    Phase ph(ctx, L, "panels");
    HIPCHK(estimator(ctx->coord ? nullptr : S.Sk, sk_dt(ctx), ctx->coord ? S.C : nullptr, ctx->V, mdt, np, ctx->n,
                     ctx->q, scale, L.red, ctx->est, ctx->status, L.s, ctx->part ? S.ht : nullptr));
    panel_times_small(ctx, L, ctx->V, mdt, ctx->Ginv, ctx->W, mdt, -1.0);  // Q^T = -T^T G^-1
    if (ctx->part) {  // (L+^T A L+)_jj
      Phase pw(ctx, L, "weights");
      HIPCHK(part_weights(ctx->V, ctx->W, mdt, np, ctx->n, ctx->q, S.C, ctx->tw, L.s));
    }
    if (ctx->coord) {
      HIPCHK(coord_add_rows(ctx->W, mdt, np, S.C, ctx->q, ctx->Z, qp, L.s));  // + E_C L_G^-1
    } else {
      small_small(ctx, L, S.Z, true, ctx->Z, ctx->Mq);  // Mq = L_M^-T L_G^-1
      panel_times_small(ctx, L, S.Sk, sk_dt(ctx), ctx->Mq, ctx->W, mdt, 1.0, ctx->W, mdt, 1.0);
    }
  }
  Phase ph(ctx, L, "update", true);  // L += S Q
  if (ctx->mixed) {
    const int64_t plane = np * qp;
    __bf16* shi = ctx->planes;
    __bf16* qhi = ctx->planes + 2 * plane;
    HIPCHK(pack_split2((const float*)ctx->Sa, np, np, qp, shi, shi + plane, qp, 0, L.s, upd_panel_tile(ctx)));
    HIPCHK(pack_split2((const float*)ctx->W, np, np, qp, qhi, qhi + plane, qp, 0, L.s, upd_panel_tile(ctx)));
    MixedGemm mg;
    GemmArgs& g = mg.g;
    g.M = np; g.N = np; g.K = qp;
    g.A = shi; g.lda = qp; g.a_plane = plane;
    g.B = qhi; g.ldb = qp; g.b_plane = plane;
    g.epi = EPI_ADDROW; g.C = ctx->X; g.ldc = np; g.c2 = 1.0;
    g.tiles = ctx->tiles; g.ntiles = ctx->ntiles; g.bn = bf16_square_tile(np, g.K, g.epi);
    mg.a_kind = OK_BF16_KC; mg.b_kind = OK_BF16_KC; mg.na = 2; mg.nb = 2; mg.pmax = 1;
    bf_gemm(ctx, L, mg);
  } else {
    GemmArgs g;
    g.M = np; g.N = np; g.K = qp;
    g.A = ctx->Sa; g.lda = np; g.a_dt = DT_F64; g.a_kc = false;
    g.B = ctx->W; g.ldb = np; g.b_dt = DT_F64; g.b_kc = false;
    g.epi = EPI_ADDROW; g.C = ctx->X; g.ldc = np; g.c_dt = DT_F64; g.c2 = 1.0;
    g.tiles = ctx->tiles; g.ntiles = ctx->ntiles;
    f64_gemm(ctx, L, g);
  }
}

// Partition weights (L^T A L)_jj of AdaRBFGS for an L the caller set: block by block,
// P = L I_{:C} (gathered), Q = A P (the step's product), t_C = column dots of P and Q;
// n^3 flops in all, once per rbfgs_set_state.  Uses slot 0's index buffer.
void refresh_part_weights(rbfgs_ctx* ctx) {
  const Lane& L = ctx->main;
  int32_t* C = ctx->slot[0].C;
  for (int64_t b = 0; b < ctx->n / ctx->q; ++b) {
    HIPCHK(fill_block(C, b * ctx->q, ctx->q, L.s));
    HIPCHK(gather_cols_gen(ctx->X, ctx->mdt, ctx->np, C, ctx->q, ctx->np, ctx->Sa, ctx->mdt, ctx->np, L.s));
    nn_times_panel(ctx, L, ctx->A, false, ctx->Sa, ctx->mdt, ctx->Y, 3, 2, 2);
    HIPCHK(col_dots(ctx->Sa, ctx->Y, ctx->mdt, ctx->np, ctx->n, ctx->q, C, ctx->tw, L.s));
  }
}

// One step of a comparison method of Sec. 10 on the main lane (FP64, n^3 products):
//   Newton-Schulz, eq. (Newton-Schulz): T = A X, X+ = 2 X - X T;
//   MR, eq. (MRiter): R = I - A X, P = X R, Q = (A X) R = R - R R, X+ = X + (<R, Q> / <Q, Q>) P,
//   where <R, Q> = Tr(R^T A X R) and <Q, Q> = Tr((A X R)^T A X R).
// The estimator is the exact ||I - A X_k||_F^2 of the iterate the step starts from.
void main_comparison(rbfgs_ctx* ctx) {
  const Lane& L = ctx->main;
  const int64_t np = ctx->np, n = ctx->n;
  auto square = [&](const void* Aop, const void* Bop, double* out, const char* name) {
    Phase ph(ctx, L, name, true);
    GemmArgs g;
    g.M = np; g.N = np; g.K = np;
    g.A = Aop; g.lda = np; g.a_dt = DT_F64; g.a_kc = true;
    g.B = Bop; g.ldb = np; g.b_dt = DT_F64; g.b_kc = false;
    g.epi = EPI_ROWSTORE; g.C = out; g.ldc = np; g.c_dt = DT_F64; g.c2 = 1.0;
    f64_gemm(ctx, L, g);
  };
  const int nb = sums_blocks(n);
  square(ctx->A, ctx->X, ctx->T2, "AX");  // T = A X
  if (ctx->ns) {
    HIPCHK(mat_sums(ctx->T2, nullptr, np, n, 0, L.red, L.s));
    HIPCHK(reduce_sum_scaled(L.red, nb, ctx->est, 1.0, ctx->status, L.s));
    square(ctx->X, ctx->T2, ctx->P2, "XT");  // X T
    HIPCHK(panel_axpby(ctx->X, DT_F64, 2.0, ctx->P2, DT_F64, -1.0, ctx->P2, DT_F64, np, np, np, L.s));
    double* xn = ctx->P2;  // the new iterate; the old buffer is next step's work matrix
    ctx->P2 = (double*)ctx->X;
    ctx->X = xn;
    return;
  }
  HIPCHK(mat_sums(ctx->T2, nullptr, np, n, 1, L.red, L.s));  // R = I - A X in place
  HIPCHK(reduce_sum_scaled(L.red, nb, ctx->est, 1.0, ctx->status, L.s));
  square(ctx->X, ctx->T2, ctx->P2, "XR");  // P = X R
  // Q = A X R taken as (A X) R = (I - R) R = R - R R: for ill-conditioned A the product
  // A (X R) carries errors of order ||A|| ||X|| eps that spoil alpha (on the rand-based
  // matrices of Sec. 10 MR then diverges), while (A X) R is as accurate as R itself
  square(ctx->T2, ctx->T2, ctx->Q2, "RR");
  HIPCHK(panel_axpby(ctx->T2, DT_F64, 1.0, ctx->Q2, DT_F64, -1.0, ctx->Q2, DT_F64, np, np, np, L.s));
  HIPCHK(mat_sums(ctx->T2, ctx->Q2, np, n, 2, L.red, L.s));
  HIPCHK(reduce_pairs(L.red, nb, ctx->scal, L.s));
  HIPCHK(axpy_ratio((double*)ctx->X, ctx->P2, np * np, ctx->scal, L.s));
}

// Side-lane work of iteration k, each issued once (the watermarks skip what an earlier call
// enqueued ahead): the sketch-dependent products, and the inverse part.
void issue_products(rbfgs_ctx* ctx, int64_t k) {
  if (k <= ctx->prod_hi) return;
  Slot& S = ctx->slot[k % rbfgs_ctx::NSLOT];
  if (S.released_valid) LANE_WAIT(ctx->side.s, S.released);
  side_products(ctx, k, S);
  ctx->prod_hi = k;
}
void issue_inverse(rbfgs_ctx* ctx, int64_t k) {
  if (k <= ctx->inv_hi) return;
  Slot& S = ctx->slot[k % rbfgs_ctx::NSLOT];
  LANE_WAIT(ctx->inv.s, S.g_ready);
  side_inverse(ctx, S);
  HIPCHK(hipEventRecord(S.ready, ctx->inv.s));
  ctx->inv_hi = k;
}

// This window's first products and inverse, enqueued before a window is captured into a
// graph, so that the graph starts from the state every replay starts from.
void prime_lookahead(rbfgs_ctx* ctx) {
  if (ctx->imp || ctx->ns || ctx->mr) return;
  if (ctx->prod_hi >= ctx->k + 1 && ctx->inv_hi >= ctx->k) return;
  HIPCHK(hipEventRecord(ctx->ev_begin, ctx->main.s));
  LANE_WAIT(ctx->side.s, ctx->ev_begin);
  LANE_WAIT(ctx->inv.s, ctx->ev_begin);
  issue_products(ctx, ctx->k);
  issue_products(ctx, ctx->k + 1);
  issue_inverse(ctx, ctx->k);
}

// Enqueue iterations k .. k+nsteps-1: the side lane runs up to two iterations ahead,
// the inverse lane one.  For the fixed method the side lane's products of iteration
// k+2 start once the main lane's X Y of iteration k is done, so that A S shares the
// GPU with the main lane's small q-sized kernels rather than with X Y.
void enqueue_steps(rbfgs_ctx* ctx, int64_t nsteps) {
  if (nsteps <= 0) return;
  if (ctx->ns || ctx->mr) {
    for (int64_t i = 0; i < nsteps; ++i, ++ctx->k) main_comparison(ctx);
    return;
  }
  constexpr int NS = rbfgs_ctx::NSLOT;
  if (ctx->imp) {  // each draw depends on X_k: no look-ahead, the lanes run one step at a time
    for (int64_t i = 0; i < nsteps; ++i) {
      const int64_t k = ctx->k;
      Slot& S = ctx->slot[k % NS];
      importance_draw(ctx, S, k);
      HIPCHK(hipEventRecord(ctx->ev_begin, ctx->main.s));
      LANE_WAIT(ctx->side.s, ctx->ev_begin);
      side_products(ctx, k, S);
      LANE_WAIT(ctx->inv.s, S.g_ready);
      side_inverse(ctx, S);
      HIPCHK(hipEventRecord(S.ready, ctx->inv.s));
      LANE_WAIT(ctx->main.s, S.y_ready);
      main_row(ctx, S, [] {}, [] {});
      HIPCHK(hipEventRecord(S.released, ctx->main.s));
      S.released_valid = true;
      ++ctx->k;
    }
    return;
  }
  HIPCHK(hipEventRecord(ctx->ev_begin, ctx->main.s));
  LANE_WAIT(ctx->side.s, ctx->ev_begin);
  LANE_WAIT(ctx->inv.s, ctx->ev_begin);
  auto products = [&](int64_t k) { issue_products(ctx, k); };
  auto inverse = [&](int64_t k) { issue_inverse(ctx, k); };
  const int64_t k0 = ctx->k;
  products(k0);
  if (nsteps > 1) products(k0 + 1);
  inverse(k0);
  for (int64_t i = 0; i < nsteps; ++i) {
    const int64_t k = ctx->k;
    auto ahead = [&]() {
      if (i + 2 < nsteps) products(k + 2);
      if (i + 1 < nsteps) inverse(k + 1);
    };
    Slot& S = ctx->slot[k % NS];
    if (ctx->ada) {
      ahead();
      LANE_WAIT(ctx->main.s, S.ready);
      main_adaptive(ctx, S, k);
    } else {
      LANE_WAIT(ctx->main.s, S.y_ready);
      // The side lane's products of k+2 and the inverse of k+1 are released after X Y, so
      // that A S runs beside the q-sized kernels and the update rather than beside X Y.
      // Measured at n = 16384, q = 256: releasing A S at the start of the iteration lets the
      // q-sized kernels run alone (0.30 -> 0.08 ms) but X Y beside A S takes 0.90 ms instead
      // of 0.53 (the pair moves no more bytes per second than either alone): 1.79 ms per step
      // against 1.76; releasing both only before the update was no faster.
      auto after_xy = [&]() {
        HIPCHK(hipEventRecord(ctx->ev_xy, ctx->main.s));
        LANE_WAIT(ctx->side.s, ctx->ev_xy);
        if (i + 2 < nsteps) products(k + 2);
        if (i + 1 < nsteps) inverse(k + 1);
      };
      auto before_update = [&]() {};
      if (ctx->rowv) main_row(ctx, S, after_xy, before_update);
      else main_fixed(ctx, S, after_xy, before_update);
    }
    HIPCHK(hipEventRecord(S.released, ctx->main.s));
    S.released_valid = true;
    ++ctx->k;
  }
  // the next window's first products and inverse, issued now: they run beside this window's
  // last steps and the host's stopping decision (they depend on the sketch and A only)
  const int64_t kend = ctx->k;
  products(kend);
  products(kend + 1);
  inverse(kend);
}

rbfgs_status fail(rbfgs_ctx* ctx, rbfgs_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

rbfgs_status read_status(rbfgs_ctx* ctx) {
  int st = 0;
  HIPCHK(hipStreamSynchronize(ctx->side.s));
  HIPCHK(hipStreamSynchronize(ctx->inv.s));
  HIPCHK(hipMemcpyAsync(&st, ctx->status, sizeof(int), hipMemcpyDeviceToHost, ctx->main.s));
  HIPCHK(hipStreamSynchronize(ctx->main.s));
  if (st == 3) return fail(ctx, RBFGS_E_NOT_SPD, "Cholesky of S^T A S met a non-positive pivot (A not SPD?)");
  if (st == 4) return fail(ctx, RBFGS_E_NONFINITE, "non-finite value in the iteration");
  if (st) return fail(ctx, RBFGS_E_DEVICE, "unknown device status");
  return RBFGS_OK;
}

// AdaRBFGS: unbiased estimate of ||I - A X||_F^2, X = L L^T, from PROBES Gaussian probe
// vectors g (E ||(I - A X) g||^2 = ||I - A X||_F^2), in FP64 on the stored A and L:
// W1 = L^T G, W2 = L W1, W1 = A W2, est = ||G - W1||_F^2 / PROBES (6 n^2 PROBES flops).  The
// probes come from the sketch stream at iteration 2^62 + w, outside the method's own range.
double probe_residual(rbfgs_ctx* ctx, uint64_t w) {
  const Lane& L = ctx->main;
  const int64_t np = ctx->np;
  double* G = ctx->prb;
  double* W1 = G + np * PROBES;
  double* W2 = W1 + np * PROBES;
  HIPCHK(sketch_gauss(ctx->p.seed, (int64_t)((1ull << 62) + w), ctx->n, PROBES, G, DT_F64, np, L.s));
  auto prod = [&](const void* M, bool transpose, const double* in, double* out) {
    GemmArgs g;
    g.M = np; g.N = PROBES; g.K = np;
    g.A = M; g.lda = np; g.a_dt = ctx->mdt; g.a_kc = !transpose;
    g.B = in; g.ldb = np; g.b_dt = DT_F64; g.b_kc = true;
    g.epi = EPI_COLSTORE; g.C = out; g.ldc = np; g.c_dt = DT_F64; g.c2 = 1.0;
    f64_gemm(ctx, L, g);
  };
  prod(ctx->X, true, G, W1);
  prod(ctx->X, false, W1, W2);
  prod(ctx->A, false, W2, W1);
  HIPCHK(estimator(G, DT_F64, nullptr, W1, DT_F64, np, ctx->n, PROBES, 1.0 / PROBES, L.red, ctx->est + 4, ctx->status,
                   L.s));
  double v = 0;
  HIPCHK(hipMemcpyAsync(&v, ctx->est + 4, sizeof(double), hipMemcpyDeviceToHost, L.s));
  HIPCHK(hipStreamSynchronize(L.s));
  return v;
}

// X held on its lower tiles: copy them onto the upper tiles before X is read whole.
void ensure_full_x(rbfgs_ctx* ctx) {
  if (!ctx->x_lower) return;
  HIPCHK(mirror_lower((float*)ctx->X, ctx->np, ctx->np / 128, ctx->main.s));
  ctx->x_lower = false;
}

double exact_residual(rbfgs_ctx* ctx) {
  ensure_full_x(ctx);
  const int64_t np = ctx->np;
  const Lane& L = ctx->main;
  GemmArgs g;
  g.M = np; g.N = np; g.K = np;
  g.A = ctx->A; g.lda = np; g.a_dt = ctx->mdt; g.a_kc = true;
  if (ctx->ada) {
    // B = A L (FP64, in the context's n x n scratch), then I - B L^T
    GemmArgs b = g;
    b.B = ctx->X; b.ldb = np; b.b_dt = ctx->mdt; b.b_kc = false;
    b.epi = EPI_ROWSTORE; b.C = ctx->sq; b.ldc = np; b.c_dt = DT_F64; b.c2 = 1.0;
    HIPCHK(gemm_f64(b, nullptr, L.s));
    g.A = ctx->sq; g.a_dt = DT_F64;
  }
  // Bop(k,j) = M[j][k]: X symmetric (fixed, PSB); L (adaptive, I - (A L) L^T); Z = X^T (row variants).
  // Newton-Schulz and MR: Bop(k,j) = X[k][j] (their iterates are symmetric only in exact
  // arithmetic, and on ill-conditioned A the rounding asymmetry grows)
  g.B = ctx->X; g.ldb = np; g.b_dt = ctx->mdt; g.b_kc = !(ctx->ns || ctx->mr);
  g.epi = EPI_RESID; g.red = L.red; g.nvalid = ctx->n;
  const int64_t blocks = gemm_f64_blocks(g);
  HIPCHK(gemm_f64(g, nullptr, L.s));
  HIPCHK(reduce_sum(L.red, blocks, ctx->est + 1, L.s));
  double r2 = 0;
  HIPCHK(hipMemcpyAsync(&r2, ctx->est + 1, sizeof(double), hipMemcpyDeviceToHost, L.s));
  HIPCHK(hipStreamSynchronize(L.s));
  return sqrt(r2);
}

// Mixed-precision n x n-by-n x q products take the streamed kernel (bf16 planes of the
// panel made once per product) when q is a multiple of 128 and n is large.
bool streamed_products(const rbfgs_ctx* ctx) { return ctx->mixed && ctx->qp % 128 == 0 && ctx->np >= 1024; }

void make_lane(rbfgs_ctx* ctx, Lane& L, size_t partial_bytes, size_t red_count) {
  L.partial_bytes = partial_bytes;
  L.partial = dalloc(ctx, partial_bytes);
  L.red = (double*)dalloc(ctx, red_count * sizeof(double));
  L.red_count = red_count;
  L.cwork = (double*)dalloc(ctx, chol_inv_work_doubles(ctx->q) * sizeof(double));
  if (streamed_products(ctx)) L.bsplit = (__bf16*)dalloc(ctx, (size_t)3 * ctx->np * ctx->qp * sizeof(__bf16));
}

void make_slot(rbfgs_ctx* ctx, Slot& S) {
  const int64_t np = ctx->np, qp = ctx->qp;
  const size_t es = dt_size(ctx->mdt), qq = (size_t)qp * qp * sizeof(double);
  S.Sk = dalloc(ctx, np * qp * dt_size(sk_dt(ctx)));
  S.C = (int32_t*)dalloc(ctx, qp * sizeof(int32_t));
  S.G = (double*)dalloc(ctx, qq);
  if (ctx->psb) S.G2 = (double*)dalloc(ctx, qq);
  S.Z = (double*)dalloc(ctx, qq);
  if (ctx->part || ctx->imp) S.ht = (double*)dalloc(ctx, sizeof(double));
  if (!ctx->ada) {
    S.Y = dalloc(ctx, np * qp * es);
    S.Ginv = (double*)dalloc(ctx, qq);
    if (ctx->bf16q) S.Ginv32 = (float*)dalloc(ctx, (size_t)qp * qp * sizeof(float));
    if (!ctx->coord) {
      S.U = dalloc(ctx, (ctx->mixed ? 1 : 3) * np * qp * es);
      if (ctx->mixed) S.planes = (__bf16*)dalloc(ctx, (size_t)(ctx->upd3 ? 3 : 2) * 3 * np * qp * sizeof(__bf16));
    }
  }
  if (ctx->dry) return;
  HIPCHK(hipEventCreateWithFlags(&S.y_ready, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&S.g_ready, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&S.ready, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&S.released, hipEventDisableTiming));
}

void release(rbfgs_ctx* ctx) {
  (void)hipStreamSynchronize(ctx->main.s);
  if (ctx->own_lanes && ctx->side.s) (void)hipStreamSynchronize(ctx->side.s);
  if (ctx->own_lanes && ctx->inv.s) (void)hipStreamSynchronize(ctx->inv.s);
  for (auto& r : ctx->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  for (Slot& S : ctx->slot) {
    if (S.y_ready) (void)hipEventDestroy(S.y_ready);
    if (S.g_ready) (void)hipEventDestroy(S.g_ready);
    if (S.ready) (void)hipEventDestroy(S.ready);
    if (S.released) (void)hipEventDestroy(S.released);
  }
  if (ctx->ev_begin) (void)hipEventDestroy(ctx->ev_begin);
  if (ctx->ev_xy) (void)hipEventDestroy(ctx->ev_xy);
  if (ctx->ev_g) (void)hipEventDestroy(ctx->ev_g);
  if (ctx->ev_chol) (void)hipEventDestroy(ctx->ev_chol);
  for (void* p : ctx->allocs) {
    if (ctx->pool) ctx->pool->release(p);
    else (void)hipFree(p);
  }
  if (ctx->own_lanes && ctx->side.s) (void)hipStreamDestroy(ctx->side.s);
  if (ctx->own_lanes && ctx->inv.s) (void)hipStreamDestroy(ctx->inv.s);
  delete ctx;
}

// Parameters and derived sizes of a context.
void set_params(rbfgs_ctx* ctx, const rbfgs_params& p) {
  ctx->p = p;
  if (ctx->p.check_every == 0) ctx->p.check_every = 16;
  ctx->n = p.n;
  ctx->q = p.q;
  ctx->np = (p.n + 255) / 256 * 256;
  ctx->qp = ((int64_t)p.q + 31) / 32 * 32;
  ctx->mixed = p.precision == RBFGS_MIXED;
  ctx->ada = p.variant == RBFGS_ADAPTIVE;
  ctx->psb = p.variant == RBFGS_PSB;
  ctx->kacz = p.variant == RBFGS_KACZMARZ;
  ctx->rowv = ctx->kacz || p.variant == RBFGS_AIP;
  ctx->ns = p.variant == RBFGS_NEWTON_SCHULZ;
  ctx->mr = p.variant == RBFGS_MR;
  ctx->part = p.sketch == RBFGS_SKETCH_PARTITION;
  ctx->imp = p.sketch == RBFGS_SKETCH_IMPORTANCE;
  ctx->dcoord = (p.sketch == RBFGS_SKETCH_COORD && (ctx->psb || ctx->rowv)) || ctx->imp;
  ctx->coord = (p.sketch == RBFGS_SKETCH_COORD && !ctx->dcoord) || ctx->part;
  ctx->mdt = ctx->mixed ? DT_F32 : DT_F64;
  ctx->bf16q = ctx->mixed && p.variant == RBFGS_FIXED && !ctx->coord && ctx->qp % 128 == 0;
  ctx->bf16h = ctx->bf16q && 8 * ctx->qp <= ctx->np;
  ctx->lowx = ctx->mixed && p.variant == RBFGS_FIXED && p.sketch == RBFGS_SKETCH_GAUSS && ctx->qp % 128 == 0 &&
              ctx->np >= 1024;
  ctx->upd3 = ctx->mixed && (p.variant == RBFGS_FIXED || ctx->psb) && !ctx->coord && 8 * ctx->qp > ctx->np;
}

// Every device buffer of the context (accounted only, in a dry run).
void allocate(rbfgs_ctx* ctx) {
  const int64_t np = ctx->np, qp = ctx->qp;
  const size_t es = dt_size(ctx->mdt);
  const size_t partial = std::max<size_t>((size_t)8 * np * qp * 8, (size_t)128 * qp * qp * sizeof(double));
  const size_t red = (size_t)std::max<int64_t>(4096, (np / 32) * (np / 32) + 16);
  make_lane(ctx, ctx->main, partial, red);
  make_lane(ctx, ctx->side, partial, 4096);
  make_lane(ctx, ctx->inv, partial, 4096);
  for (Slot& S : ctx->slot) make_slot(ctx, S);
  ctx->A = dalloc(ctx, np * np * es);
  ctx->X = dalloc(ctx, np * np * es);
  ctx->pos = (int32_t*)dalloc(ctx, np * sizeof(int32_t));
  if (!ctx->dry) HIPCHK(hipMemsetAsync(ctx->pos, 0xff, np * sizeof(int32_t), ctx->main.s));  // -1
  ctx->V = dalloc(ctx, np * qp * es);
  ctx->W = dalloc(ctx, np * qp * es);
  if (ctx->ada) {
    ctx->Sa = dalloc(ctx, np * qp * es);
    ctx->Y = dalloc(ctx, np * qp * es);
    if (ctx->mixed) ctx->planes = (__bf16*)dalloc(ctx, (size_t)4 * np * qp * sizeof(__bf16));
  }
  if (ctx->rowv && ctx->mixed) ctx->planes = (__bf16*)dalloc(ctx, (size_t)2 * np * qp * sizeof(__bf16));
  if (ctx->ns || ctx->mr) {
    ctx->T2 = (double*)dalloc(ctx, (size_t)np * np * sizeof(double));
    ctx->P2 = (double*)dalloc(ctx, (size_t)np * np * sizeof(double));
    if (ctx->mr) ctx->Q2 = (double*)dalloc(ctx, (size_t)np * np * sizeof(double));
  }
  ctx->scal = (double*)dalloc(ctx, 8 * sizeof(double));
  if (ctx->part || ctx->imp) ctx->tw = (double*)dalloc(ctx, np * sizeof(double));
  if (ctx->imp) {
    ctx->BA = (double*)dalloc(ctx, (size_t)(ctx->n / ctx->q) * qp * qp * sizeof(double));
    ctx->ipart_cap = block_weights_workspace(ctx->n, (int)ctx->q);
    ctx->ipart = (double*)dalloc(ctx, (size_t)ctx->ipart_cap * sizeof(double));
    ctx->Pz = dalloc(ctx, np * qp * es);
    if (!ctx->dry) HIPCHK(hipMemsetAsync(ctx->Pz, 0, np * qp * es, ctx->main.s));  // pad columns stay 0
  }
  if (!ctx->ada && ctx->coord) ctx->R = dalloc(ctx, qp * np * es);
  const size_t qq = (size_t)qp * qp * sizeof(double);
  ctx->G = (double*)dalloc(ctx, qq);
  ctx->H = (double*)dalloc(ctx, qq);
  if (ctx->bf16h) ctx->H32 = (float*)dalloc(ctx, (size_t)qp * qp * sizeof(float));
  ctx->Ginv = (double*)dalloc(ctx, qq);
  ctx->Z = (double*)dalloc(ctx, qq);
  ctx->GH = (double*)dalloc(ctx, qq);
  ctx->Mq = (double*)dalloc(ctx, qq);
  ctx->est = (double*)dalloc(ctx, 8 * sizeof(double));
  if (ctx->pool) ctx->kdev = (int64_t*)dalloc(ctx, sizeof(int64_t));
  if (ctx->ada) ctx->prb = (double*)dalloc(ctx, (size_t)3 * np * PROBES * sizeof(double));
  ctx->status = (int*)dalloc(ctx, sizeof(int));
  if (ctx->ada) ctx->sq = dalloc(ctx, (size_t)np * np * sizeof(double));
  else if (ctx->rowv) ctx->sq = dalloc(ctx, (size_t)np * np * es);
  ctx->stage_bytes = std::min<size_t>((size_t)np * np * sizeof(double), (size_t)32 << 20);
  ctx->stage = dalloc(ctx, ctx->stage_bytes);
  {  // tile order of the n x n update: lower triangle (symmetric X) or full square (L, row variants)
    const bool full = ctx->ada || ctx->rowv;
    const int epi = full ? EPI_ADDROW : EPI_SYMUPD;
    const int T = (int)(np / (ctx->mixed ? bf16_square_tile(np, full ? qp : 2 * qp, epi) : 128));
    std::vector<int2> order((size_t)make_tile_order(T, SUPER_TILES, !full, nullptr));
    ctx->ntiles = make_tile_order(T, SUPER_TILES, !full, order.data());
    ctx->tiles = (int2*)dalloc(ctx, order.size() * sizeof(int2));
    if (!ctx->dry) {
      HIPCHK(hipMemcpyAsync(ctx->tiles, order.data(), order.size() * sizeof(int2), hipMemcpyHostToDevice,
                            ctx->main.s));
      HIPCHK(hipStreamSynchronize(ctx->main.s));
    }
  }
}

// The stopping rule of rbfgs_invert, the part after each window of m = st.m iterations whose
// estimates sum to est_sum: the estimator trigger, the AdaRBFGS probe, the exact residual.
void invert_decide(rbfgs_ctx* ctx, rb::InvertState& st, double est_sum) {
  RocRange range("stopping_test");
  const double est = est_sum / (double)st.m;
  const double tol = st.tol;
  if (ctx->ada) {
    // the free estimate measures ||I - L^T A L||_F^2 <= ||I - A X||_F^2: only below the
    // target is the unbiased probe estimate of ||I - A X||_F^2 taken, and only below the
    // target again is the exact residual computed
    bool check = st.done >= st.next_force;
    // (the probe estimate must fall below 0.8 of the target, about one standard deviation
    // of a 64-probe estimate, so that a check rarely fails)
    if (!check && est <= st.target) check = probe_residual(ctx, (uint64_t)ctx->k) <= 0.8 * st.target;
    if (check) {
      const double r = exact_residual(ctx);
      st.resid = r / sqrt((double)ctx->n);
      if (st.resid <= tol) {
        st.result = RBFGS_OK;
        st.finished = true;
        return;
      }
      st.next_force = st.done + std::max<int64_t>(st.force_base, st.done);
    }
  } else if (est <= st.thresh || st.done >= st.next_force) {
    const double r = exact_residual(ctx);
    st.resid = r / sqrt((double)ctx->n);
    if (st.resid <= tol) {
      st.result = RBFGS_OK;
      st.finished = true;
      return;
    }
    // the estimate runs below the exact value: scale the trigger by the ratio observed
    // at this check (the latest, not the smallest: the ratio drifts as X converges)
    if (r > 0 && est > 0) st.thresh = std::min(st.target, st.target * est / (r * r));
    st.next_force = st.done + std::max<int64_t>(st.force_base, ctx->coord || ctx->dcoord ? st.done / 2 : st.done);
  }
  if (st.done >= st.max_iters) st.finished = true;  // result stays E_NOT_CONVERGED
}

}  // namespace

static rbfgs_status create_impl(const rbfgs_params* params, const void* A, int32_t a_dtype, int64_t lda,
                                int32_t a_on_device, hipStream_t stream, rb::DevicePool* pool, rbfgs_ctx** out) {
  RocRange range("rbfgs_create");
  if (!out) return RBFGS_E_INVALID_ARG;
  *out = nullptr;
  if (!params || !A) return RBFGS_E_INVALID_ARG;
  const rbfgs_params& p = *params;
  if (p.n < 1 || p.q < 1 || p.q > p.n || p.q > 1024 || lda < p.n || (a_dtype != RBFGS_F32 && a_dtype != RBFGS_F64) ||
      (p.sketch < RBFGS_SKETCH_GAUSS || p.sketch > RBFGS_SKETCH_IMPORTANCE) ||
      (p.sketch == RBFGS_SKETCH_PARTITION &&
       ((p.variant != RBFGS_FIXED && p.variant != RBFGS_ADAPTIVE) || p.n % p.q != 0)) ||
      (p.sketch == RBFGS_SKETCH_IMPORTANCE && (p.variant != RBFGS_KACZMARZ || p.n % p.q != 0)) ||
      (p.variant < RBFGS_FIXED || p.variant > RBFGS_MR) ||
      ((p.variant == RBFGS_NEWTON_SCHULZ || p.variant == RBFGS_MR) && p.precision != RBFGS_FP64) ||
      (p.precision != RBFGS_FP64 && p.precision != RBFGS_MIXED) || p.check_every < 0 || p.n > (1ll << 20))
    return RBFGS_E_INVALID_ARG;
  rbfgs_ctx* ctx = new rbfgs_ctx();
  set_params(ctx, p);
  ctx->main.s = stream;
  ctx->pool = pool;
  ctx->own_lanes = pool == nullptr;
  try {
    HIPCHK(hipGetDevice(&ctx->device));
    if (ctx->own_lanes) {
      HIPCHK(hipStreamCreateWithFlags(&ctx->side.s, hipStreamNonBlocking));  // default priority
      HIPCHK(hipStreamCreateWithFlags(&ctx->inv.s, hipStreamNonBlocking));   // default priority
    } else {  // serving: the lanes share the slot's stream
      ctx->side.s = stream;
      ctx->inv.s = stream;
    }
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_begin, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_xy, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_g, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_chol, hipEventDisableTiming));
    allocate(ctx);
    const int64_t np = ctx->np;
    // copy A (n x n, lda) into the padded np x np buffer, converting its type (a host A
    // in row chunks through the staging buffer), then check the stored matrix
    const int sdt = a_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
    const size_t ses = dt_size(sdt);
    if (a_on_device) {
      HIPCHK(copy_convert(A, sdt, lda, ctx->A, ctx->mdt, np, p.n, p.n, ctx->main.s));
    } else {
      const size_t row = (size_t)p.n * ses;
      const int64_t chunk = std::max<int64_t>(1, (int64_t)(ctx->stage_bytes / row));
      for (int64_t r0 = 0; r0 < p.n; r0 += chunk) {
        const int64_t rows = std::min(chunk, p.n - r0);
        HIPCHK(hipMemcpy2DAsync(ctx->stage, row, (const char*)A + (size_t)r0 * lda * ses, (size_t)lda * ses, row,
                                (size_t)rows, hipMemcpyHostToDevice, ctx->main.s));
        HIPCHK(copy_convert(ctx->stage, sdt, p.n, (char*)ctx->A + (size_t)r0 * np * dt_size(ctx->mdt), ctx->mdt, np,
                            rows, p.n, ctx->main.s));
        HIPCHK(hipStreamSynchronize(ctx->main.s));
      }
    }
    int* flag = ctx->status;
    const bool need_sym = p.variant != RBFGS_KACZMARZ;  // Kaczmarz takes any invertible A
    HIPCHK(check_sym_finite(ctx->A, ctx->mdt, np, p.n, flag, ctx->main.s, need_sym));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->main.s));
    HIPCHK(hipStreamSynchronize(ctx->main.s));
    if (bad) {
      release(ctx);
      return RBFGS_E_INVALID_ARG;
    }
    if (ctx->ns) {  // X_0 = 0.99 A^T / rho^2(A), rho by the power method (Sec. 10)
      double* v = (double*)ctx->T2;
      HIPCHK(power_norm((const double*)ctx->A, np, p.n, POWER_STEPS, v, v + np, ctx->scal, ctx->main.s));
      HIPCHK(ns_start((const double*)ctx->A, np, p.n, ctx->scal, (double*)ctx->X, ctx->main.s));
      HIPCHK(hipMemsetAsync(ctx->T2, 0, (size_t)2 * np * sizeof(double), ctx->main.s));
    } else if (ctx->mr) {  // X_0 = (Tr A / Tr(A A^T)) I (Sec. 10)
      HIPCHK(mat_sums((double*)ctx->A, nullptr, np, p.n, 3, ctx->main.red, ctx->main.s));
      HIPCHK(reduce_pairs(ctx->main.red, sums_blocks(p.n), ctx->scal, ctx->main.s));
      HIPCHK(scaled_identity((double*)ctx->X, np, p.n, ctx->scal, ctx->main.s));
    } else {
      HIPCHK(set_identity(ctx->X, ctx->mdt, np, p.n, ctx->main.s));
    }
    if (ctx->part) HIPCHK(diag_weights(ctx->A, ctx->mdt, np, p.n, ctx->tw, ctx->main.s));  // L_0 = I
    if (ctx->imp)  // (A A^T)_{C_i C_i} of every block, once
      for (int64_t b = 0; b < p.n / p.q; ++b)
        row_block_gram(ctx, ctx->main, ctx->A, b, ctx->BA + b * ctx->qp * ctx->qp);
    const double nanv = NAN;
    HIPCHK(hipMemcpyAsync(ctx->est, &nanv, sizeof(double), hipMemcpyHostToDevice, ctx->main.s));
    HIPCHK(hipStreamSynchronize(ctx->main.s));
  } catch (const Fail& f) {
    release(ctx);
    return f.st;
  }
  *out = ctx;
  return RBFGS_OK;
}

rbfgs_status rbfgs_create_pooled(const rbfgs_params* params, const void* A, int32_t a_dtype, int64_t lda,
                                 int32_t a_on_device, hipStream_t stream, rb::DevicePool* pool, rbfgs_ctx** out) {
  if (!pool) return RBFGS_E_INVALID_ARG;
  return create_impl(params, A, a_dtype, lda, a_on_device, stream, pool, out);
}

void rbfgs_invert_begin(rbfgs_ctx* ctx, rb::InvertState& st, double tol, int64_t max_iters) {
  st = rb::InvertState();
  st.tol = tol;
  st.max_iters = max_iters;
  st.target = tol * tol * (double)ctx->n;  // estimator target for ||I - XA||_F^2
  st.thresh = st.target;
  // a check is also forced after a gap without one, so that a trigger lowered by an
  // unluckily small estimate cannot lock out the test: max(64 windows, iterations so far)
  // for Gaussian sketches; max(16 windows, half the iterations so far) for coordinate and
  // partition sketches, whose estimates are heavy-tailed when the residual sits in few
  // columns (a typical window mean is then far below the true mean)
  // (AdaRBFGS, triggered by an unbiased estimate of the decided quantity: 256 windows)
  st.force_base = (ctx->ada ? 256 : ctx->coord || ctx->dcoord ? 16 : 64) * (int64_t)ctx->p.check_every;
  st.next_force = st.force_base;
  st.finished = max_iters <= 0;
}

rbfgs_status rbfgs_invert_enqueue(rbfgs_ctx* ctx, rb::InvertState& st, double* host_est, int* host_status,
                                  hipEvent_t done) {
  const hipStream_t s = ctx->main.s;
  try {
    st.m = std::min<int64_t>(ctx->p.check_every, st.max_iters - st.done);
    // full windows of a serving context with a Gaussian sketch run as one replayed graph: all
    // lanes share one stream, and a window of a multiple of 3 steps starts at a multiple of 3,
    // so every window visits the sketch slots in the same order
    const bool graph = ctx->kdev && ctx->p.sketch == RBFGS_SKETCH_GAUSS && !ctx->prof &&
                       (ctx->p.variant == RBFGS_FIXED || ctx->p.variant == RBFGS_ADAPTIVE) &&
                       ctx->p.check_every % 3 == 0 && st.m == ctx->p.check_every && ctx->k % 3 == 0;
    if (!graph) {
      RocRange range("window");
      HIPCHK(fill_f64(ctx->est + 2, 1, 0.0, s));
      enqueue_steps(ctx, st.m);
    } else if (!ctx->gexec) {
      RocRange range("window.capture");
      // the graph starts from the state every replay starts from: this window's first products
      // and inverse already enqueued (by the previous window, or here)
      prime_lookahead(ctx);
      const int64_t k0 = ctx->k;
      HIPCHK(hipMemsetAsync(ctx->kdev, 0, sizeof(int64_t), s));
      HIPCHK(add_i64(ctx->kdev, k0, s));
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      ctx->kcap0 = k0;
      try {
        HIPCHK(fill_f64(ctx->est + 2, 1, 0.0, s));
        enqueue_steps(ctx, st.m);
        HIPCHK(add_i64(ctx->kdev, st.m, s));
      } catch (const Fail&) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(s, &g);
        if (g) (void)hipGraphDestroy(g);
        ctx->kcap0 = -1;
        throw;
      }
      ctx->kcap0 = -1;
      HIPCHK(hipStreamEndCapture(s, &ctx->graph));
      HIPCHK(hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
      HIPCHK(hipGraphLaunch(ctx->gexec, s));
    } else {
      RocRange range("window.replay");
      HIPCHK(hipGraphLaunch(ctx->gexec, s));
      ctx->k += st.m;
      ctx->prod_hi += st.m;  // the graph ends by enqueueing the next window's side-lane work
      ctx->inv_hi += st.m;
    }
    st.done += st.m;
    HIPCHK(hipMemcpyAsync(host_est, ctx->est + 2, sizeof(double), hipMemcpyDeviceToHost, ctx->main.s));
    HIPCHK(hipMemcpyAsync(host_status, ctx->status, sizeof(int), hipMemcpyDeviceToHost, ctx->main.s));
    HIPCHK(hipEventRecord(done, ctx->main.s));
  } catch (const Fail& f) {
    return f.st;
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_invert_after(rbfgs_ctx* ctx, rb::InvertState& st, double est_sum, int status) {
  if (status) {
    st.finished = true;
    st.result = status == 3 ? RBFGS_E_NOT_SPD : status == 4 ? RBFGS_E_NONFINITE : RBFGS_E_DEVICE;
    return st.result;
  }
  try {
    invert_decide(ctx, st, est_sum);
  } catch (const Fail& f) {
    st.finished = true;
    st.result = f.st;
  }
  return RBFGS_OK;
}

extern "C" {

rbfgs_status rbfgs_create(const rbfgs_params* params, const void* A, int32_t a_dtype, int64_t lda,
                          int32_t a_on_device, void* hip_stream, rbfgs_ctx** out) {
  return create_impl(params, A, a_dtype, lda, a_on_device, (hipStream_t)hip_stream, nullptr, out);
}

rbfgs_status rbfgs_step(rbfgs_ctx* ctx, int64_t nsteps) {
  if (!ctx || nsteps < 0) return RBFGS_E_INVALID_ARG;
  try {
    enqueue_steps(ctx, nsteps);
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
    HIPCHK(hipMemcpyAsync(est_out, ctx->est, sizeof(double), hipMemcpyDeviceToHost, ctx->main.s));
    HIPCHK(hipStreamSynchronize(ctx->main.s));
  } catch (const Fail& f) {
    return f.st;
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_invert(rbfgs_ctx* ctx, double tol, int64_t max_iters, int64_t* iters_out, double* resid_out) {
  if (!ctx || !(tol > 0) || max_iters < 0) return RBFGS_E_INVALID_ARG;
  rb::InvertState st;
  rbfgs_invert_begin(ctx, st, tol, max_iters);
  rbfgs_status result = RBFGS_E_NOT_CONVERGED;
  try {
    while (!st.finished) {
      RocRange range("window");
      double est = 0;
      HIPCHK(hipMemsetAsync(ctx->est + 2, 0, sizeof(double), ctx->main.s));
      enqueue_steps(ctx, st.m = std::min<int64_t>(ctx->p.check_every, st.max_iters - st.done));
      st.done += st.m;
      rbfgs_status s = read_status(ctx);
      if (s != RBFGS_OK) {
        st.finished = true;
        st.result = s;
        break;
      }
      HIPCHK(hipMemcpyAsync(&est, ctx->est + 2, sizeof(double), hipMemcpyDeviceToHost, ctx->main.s));
      HIPCHK(hipStreamSynchronize(ctx->main.s));
      invert_decide(ctx, st, est);
    }
    result = st.result;
  } catch (const Fail& f) {
    result = f.st;
  }
  if (iters_out) *iters_out = st.done;
  if (resid_out) *resid_out = st.resid;
  if (result == RBFGS_E_NOT_CONVERGED) ctx->err = "max_iters reached above tolerance";
  return result;
}

// n x n block of src (element type src_dt, leading dimension lds) to the caller's dst,
// converted to d_dtype; a host dst is filled in row chunks through the context's staging.
static rbfgs_status copy_out(rbfgs_ctx* ctx, const void* src, int src_dt, int64_t lds, void* dst, int32_t d_dtype,
                             int64_t ldd, int32_t on_device) {
  const int ddt = d_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
  const int64_t n = ctx->n;
  hipStream_t s = ctx->main.s;
  if (on_device) {
    HIPCHK(copy_convert(src, src_dt, lds, dst, ddt, ldd, n, n, s));
    HIPCHK(hipStreamSynchronize(s));
    return RBFGS_OK;
  }
  const size_t row = (size_t)n * dt_size(ddt);
  const int64_t chunk = std::max<int64_t>(1, (int64_t)(ctx->stage_bytes / row));
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int64_t rows = std::min(chunk, n - r0);
    HIPCHK(copy_convert((const char*)src + (size_t)r0 * lds * dt_size(src_dt), src_dt, lds, ctx->stage, ddt, n, rows,
                        n, s));
    HIPCHK(hipMemcpy2DAsync((char*)dst + (size_t)r0 * ldd * dt_size(ddt), (size_t)ldd * dt_size(ddt), ctx->stage, row,
                            row, (size_t)rows, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_get_x(rbfgs_ctx* ctx, void* X, int32_t x_dtype, int64_t ldx, int32_t on_device) {
  if (!ctx || !X || ldx < ctx->n || (x_dtype != RBFGS_F32 && x_dtype != RBFGS_F64)) return RBFGS_E_INVALID_ARG;
  try {
    rbfgs_status st = read_status(ctx);
    if (st != RBFGS_OK) return st;
    if (ctx->rowv) {  // the context holds X^T
      HIPCHK(copy_transpose(ctx->X, ctx->mdt, ctx->np, ctx->sq, ctx->mdt, ctx->np, ctx->np, ctx->np, ctx->main.s));
      return copy_out(ctx, ctx->sq, ctx->mdt, ctx->np, X, x_dtype, ldx, on_device);
    }
    if (!ctx->ada) {
      ensure_full_x(ctx);
      return copy_out(ctx, ctx->X, ctx->mdt, ctx->np, X, x_dtype, ldx, on_device);
    }
    const int64_t np = ctx->np;
    GemmArgs g;
    g.M = np; g.N = np; g.K = np;
    g.A = ctx->X; g.lda = np; g.a_dt = ctx->mdt; g.a_kc = true;
    g.B = ctx->X; g.ldb = np; g.b_dt = ctx->mdt; g.b_kc = true;  // Bop(k,j) = L[j][k]
    g.epi = EPI_ROWSTORE; g.C = ctx->sq; g.ldc = np; g.c_dt = DT_F64; g.c2 = 1.0;
    HIPCHK(gemm_f64(g, nullptr, ctx->main.s));
    return copy_out(ctx, ctx->sq, DT_F64, np, X, x_dtype, ldx, on_device);
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
    HIPCHK(hipStreamSynchronize(ctx->side.s));
    HIPCHK(hipStreamSynchronize(ctx->inv.s));
    if (on_device) {
      if (ctx->rowv) HIPCHK(copy_transpose(M, sdt, ldm, ctx->X, ctx->mdt, ctx->np, n, n, ctx->main.s));  // X^T
      else HIPCHK(copy_convert(M, sdt, ldm, ctx->X, ctx->mdt, ctx->np, n, n, ctx->main.s));
    } else {
      // row chunks through the staging buffer
      const size_t row = (size_t)n * dt_size(sdt);
      const int64_t chunk = std::max<int64_t>(1, (int64_t)(ctx->stage_bytes / row));
      for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t rows = std::min(chunk, n - r0);
        HIPCHK(hipMemcpy2DAsync(ctx->stage, row, (const char*)M + (size_t)r0 * ldm * dt_size(sdt),
                                (size_t)ldm * dt_size(sdt), row, (size_t)rows, hipMemcpyHostToDevice, ctx->main.s));
        if (ctx->rowv)  // rows r0.. of M are columns r0.. of the stored X^T
          HIPCHK(copy_transpose(ctx->stage, sdt, n, (char*)ctx->X + (size_t)r0 * dt_size(ctx->mdt), ctx->mdt, ctx->np,
                                rows, n, ctx->main.s));
        else
          HIPCHK(copy_convert(ctx->stage, sdt, n, (char*)ctx->X + (size_t)r0 * ctx->np * dt_size(ctx->mdt), ctx->mdt,
                              ctx->np, rows, n, ctx->main.s));
        HIPCHK(hipStreamSynchronize(ctx->main.s));
      }
    }
    ctx->x_lower = false;  // written whole
    HIPCHK(hipMemsetAsync(ctx->status, 0, sizeof(int), ctx->main.s));
    if (ctx->part && ctx->ada) refresh_part_weights(ctx);
    HIPCHK(hipStreamSynchronize(ctx->main.s));
    ctx->k = k;
    ctx->prod_hi = ctx->inv_hi = k - 1;  // nothing of the new iterations is enqueued
  } catch (const Fail& f) {
    return f.st;
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_get_weights(rbfgs_ctx* ctx, double* out) {
  if (!ctx || !out || !(ctx->part || ctx->imp)) return RBFGS_E_INVALID_ARG;
  try {
    rbfgs_status st = read_status(ctx);
    if (st != RBFGS_OK) return st;
    HIPCHK(hipMemcpyAsync(out, ctx->tw, (size_t)ctx->n * sizeof(double), hipMemcpyDeviceToHost, ctx->main.s));
    HIPCHK(hipStreamSynchronize(ctx->main.s));
  } catch (const Fail& f) {
    return f.st;
  }
  return RBFGS_OK;
}

rbfgs_status rbfgs_sample_partition(const double* t_dev, int64_t n, int32_t q, uint64_t seed, int64_t k,
                                    int32_t* idx_dev, double* ht_dev, void* hip_stream) {
  if (!t_dev || !idx_dev || n < 1 || q < 1 || q > n || n % q != 0 || k < 0 || n > (1ll << 20))
    return RBFGS_E_INVALID_ARG;
  hipError_t e = sample_partition(t_dev, n, q, seed, k, idx_dev, ht_dev, nullptr, (hipStream_t)hip_stream);
  return e == hipSuccess ? RBFGS_OK : RBFGS_E_DEVICE;
}

rbfgs_status rbfgs_get_iter(const rbfgs_ctx* ctx, int64_t* k_out) {
  if (!ctx || !k_out) return RBFGS_E_INVALID_ARG;
  *k_out = ctx->k;
  return RBFGS_OK;
}

rbfgs_status rbfgs_footprint(const rbfgs_params* params, int64_t* bytes_out) {
  if (!params || !bytes_out) return RBFGS_E_INVALID_ARG;
  const rbfgs_params& p = *params;
  if (p.n < 1 || p.q < 1 || p.q > p.n || p.q > 1024 || p.n > (1ll << 20)) return RBFGS_E_INVALID_ARG;
  rbfgs_ctx ctx;
  ctx.dry = true;
  set_params(&ctx, p);
  try {
    allocate(&ctx);
  } catch (const Fail& f) {
    return f.st;
  }
  *bytes_out = ctx.bytes;
  return RBFGS_OK;
}

void rbfgs_destroy(rbfgs_ctx* ctx) {
  if (ctx) release(ctx);
}

rbfgs_status rbfgs_profile(rbfgs_ctx* ctx, int32_t enable) {
  if (!ctx) return RBFGS_E_INVALID_ARG;
  try {
    prof_flush(ctx);
    ctx->prof_acc.clear();
  } catch (const Fail& f) {
    return f.st;
  }
  if (enable < 0 || enable > 2) return RBFGS_E_INVALID_ARG;
  ctx->prof = enable;
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

rbfgs_status rbfgs_pcg(rbfgs_ctx* ctx, const void* b, int32_t b_dtype, int32_t b_on_device, void* x, int32_t x_dtype,
                       int32_t x_on_device, int32_t precond, double tol, int64_t max_iters, int64_t* iters_out,
                       double* relres_out) {
  if (!ctx || !b || !x || (b_dtype != RBFGS_F32 && b_dtype != RBFGS_F64) || (x_dtype != RBFGS_F32 && x_dtype != RBFGS_F64) ||
      (precond != 0 && precond != 1) || !(tol > 0) || max_iters < 0)
    return RBFGS_E_INVALID_ARG;
  // A must be SPD; with the preconditioner, X must be too (fixed RBFGS, AdaRBFGS)
  if (ctx->kacz || ctx->psb || (precond == 1 && !(ctx->p.variant == RBFGS_FIXED || ctx->ada)))
    return RBFGS_E_INVALID_ARG;
  if (iters_out) *iters_out = 0;
  if (relres_out) *relres_out = NAN;
  void* work = nullptr;
  void* staging = nullptr;
  try {
    rbfgs_status st = read_status(ctx);
    if (st != RBFGS_OK) return st;
    if (precond) ensure_full_x(ctx);
    const int64_t n = ctx->n, np = ctx->np;
    hipStream_t s = ctx->main.s;
    const int mdt = ctx->mdt;
    HIPCHK(hipMalloc(&work, (size_t)(7 + GEMV_T_CHUNKS) * n * sizeof(double) + 8 * sizeof(double)));
    double* xv = (double*)work;
    double *r = xv + n, *z = r + n, *p = z + n, *Ap = p + n, *t = Ap + n, *part = t + 2 * n;
    double* sc = part + (size_t)GEMV_T_CHUNKS * n;  // [p.Ap, r.r, r.z (two slots)]
    const int sdt = b_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
    const void* bsrc = b;
    if (!b_on_device) {
      HIPCHK(hipMalloc(&staging, (size_t)n * dt_size(sdt)));
      HIPCHK(hipMemcpyAsync(staging, b, (size_t)n * dt_size(sdt), hipMemcpyHostToDevice, s));
      bsrc = staging;
    }
    HIPCHK(copy_convert(bsrc, sdt, n, r, DT_F64, n, 1, n, s));  // r_0 = b (x_0 = 0)
    HIPCHK(hipMemsetAsync(xv, 0, (size_t)n * sizeof(double), s));
    auto apply_m = [&](const double* in, double* out) {
      if (precond == 0) {
        HIPCHK(hipMemcpyAsync(out, in, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
      } else if (ctx->ada) {  // X = L L^T: out = L (L^T in)
        HIPCHK(gemv(ctx->X, mdt, np, n, true, in, t, part, s));
        HIPCHK(gemv(ctx->X, mdt, np, n, false, t, out, part, s));
      } else {
        HIPCHK(gemv(ctx->X, mdt, np, n, false, in, out, part, s));
      }
    };
    double host[2] = {0, 0};
    HIPCHK(dot(r, r, n, sc + 1, s));
    HIPCHK(hipMemcpyAsync(host, sc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double nb = std::sqrt(host[0]);
    double rel = nb > 0 ? 1.0 : 0.0;
    int64_t k = 0;
    bool done = !(nb > 0) || rel <= tol;
    if (!std::isfinite(nb)) {
      (void)hipFree(work);
      if (staging) (void)hipFree(staging);
      return RBFGS_E_INVALID_ARG;
    }
    if (!done) {
      apply_m(r, z);
      HIPCHK(hipMemcpyAsync(p, z, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(dot(r, z, n, sc + 2, s));
    }
    while (!done && k < max_iters) {
      const int cur = 2 + (int)(k & 1), nxt = 2 + (int)((k + 1) & 1);
      HIPCHK(gemv(ctx->A, mdt, np, n, false, p, Ap, part, s));
      HIPCHK(dot(p, Ap, n, sc, s));
      HIPCHK(cg_xr(xv, r, p, Ap, n, sc, cur, 0, s));
      apply_m(r, z);
      HIPCHK(dot(r, z, n, sc + nxt, s));
      HIPCHK(cg_p(p, z, n, sc, nxt, cur, s));
      ++k;
      if (k % 8 == 0 || k == max_iters) {  // the stopping test reads ||r|| every 8 iterations
        HIPCHK(dot(r, r, n, sc + 1, s));
        HIPCHK(hipMemcpyAsync(host, sc + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        rel = std::sqrt(host[0]) / nb;
        if (!std::isfinite(rel)) {
          (void)hipFree(work);
          if (staging) (void)hipFree(staging);
          return fail(ctx, RBFGS_E_NONFINITE, "non-finite residual in PCG");
        }
        done = rel <= tol;
      }
    }
    // x out (converted), on the host or the device
    const int ddt = x_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
    if (x_on_device) {
      HIPCHK(copy_convert(xv, DT_F64, n, x, ddt, n, 1, n, s));
    } else {
      HIPCHK(copy_convert(xv, DT_F64, n, t, ddt, n, 1, n, s));  // t is free now
      HIPCHK(hipMemcpyAsync(x, t, (size_t)n * dt_size(ddt), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    void* w = work;
    work = nullptr;
    HIPCHK(hipFree(w));
    void* st_buf = staging;
    staging = nullptr;
    if (st_buf) HIPCHK(hipFree(st_buf));
    if (iters_out) *iters_out = k;
    if (relres_out) *relres_out = rel;
    return done ? RBFGS_OK : RBFGS_E_NOT_CONVERGED;
  } catch (const Fail& f) {
    (void)hipStreamSynchronize(ctx->main.s);
    if (work) (void)hipFree(work);
    if (staging) (void)hipFree(staging);
    return f.st;
  }
}

// Ridge Hessian scale * B^T B + lambda I (eq. ridgeMatrix) in FP64: B copied into a
// zero-padded FP64 buffer (rows to a multiple of 16, columns to a multiple of 128), the
// output initialised to lambda I and updated by the FP64-MFMA symmetric product on its
// lower tiles (mirrored), then the n x n block converted into the caller's buffer.
rbfgs_status rbfgs_ridge_hessian(const void* B, int32_t b_dtype, int64_t m, int64_t n, int64_t ldb,
                                 int32_t b_on_device, double scale, double lambda, void* A, int32_t a_dtype,
                                 int64_t lda, int32_t a_on_device, void* hip_stream) {
  if (!B || !A || m < 1 || n < 1 || n > (1ll << 20) || m > (1ll << 24) || ldb < n || lda < n ||
      (b_dtype != RBFGS_F32 && b_dtype != RBFGS_F64) || (a_dtype != RBFGS_F32 && a_dtype != RBFGS_F64) ||
      !std::isfinite(scale) || !std::isfinite(lambda))
    return RBFGS_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t np = (n + 127) / 128 * 128, mp = (m + 15) / 16 * 16;
  const int sdt = b_dtype == RBFGS_F32 ? DT_F32 : DT_F64, ddt = a_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
  void *Bh = nullptr, *Bp = nullptr, *Ap = nullptr, *Ah = nullptr;
  double* sc = nullptr;
  rbfgs_status st = RBFGS_OK;
  auto chk = [&](hipError_t e) {
    if (e != hipSuccess && st == RBFGS_OK) st = e == hipErrorOutOfMemory ? RBFGS_E_OOM : RBFGS_E_DEVICE;
    return e == hipSuccess;
  };
  const double host_sc[2] = {lambda, 1.0};
  do {
    const void* Bsrc = B;
    if (!b_on_device) {
      if (!chk(hipMalloc(&Bh, (size_t)m * ldb * dt_size(sdt)))) break;
      if (!chk(hipMemcpyAsync(Bh, B, (size_t)m * ldb * dt_size(sdt), hipMemcpyHostToDevice, s))) break;
      Bsrc = Bh;
    }
    if (!chk(hipMalloc(&Bp, (size_t)mp * np * sizeof(double)))) break;
    if (!chk(hipMalloc(&Ap, (size_t)np * np * sizeof(double)))) break;
    if (!chk(hipMalloc((void**)&sc, 2 * sizeof(double)))) break;
    if (!chk(hipMemsetAsync(Bp, 0, (size_t)mp * np * sizeof(double), s))) break;
    if (!chk(hipMemsetAsync(Ap, 0, (size_t)np * np * sizeof(double), s))) break;
    if (!chk(hipMemcpyAsync(sc, host_sc, sizeof(host_sc), hipMemcpyHostToDevice, s))) break;
    if (!chk(copy_convert(Bsrc, sdt, ldb, Bp, DT_F64, np, m, n, s))) break;
    if (!chk(scaled_identity((double*)Ap, np, n, sc, s))) break;  // lambda I
    GemmArgs g;
    g.M = np; g.N = np; g.K = mp;
    g.A = Bp; g.lda = np; g.a_dt = DT_F64; g.a_kc = false;  // Aop(i, k) = B[k][i]
    g.B = Bp; g.ldb = np; g.b_dt = DT_F64; g.b_kc = false;  // Bop(k, j) = B[k][j]
    g.epi = EPI_SYMUPD; g.C = Ap; g.ldc = np; g.c_dt = DT_F64; g.c2 = scale;
    if (!chk(gemm_f64(g, nullptr, s))) break;
    if (a_on_device) {
      if (!chk(copy_convert(Ap, DT_F64, np, A, ddt, lda, n, n, s))) break;
    } else {
      if (!chk(hipMalloc(&Ah, (size_t)n * lda * dt_size(ddt)))) break;
      if (!chk(copy_convert(Ap, DT_F64, np, Ah, ddt, lda, n, n, s))) break;
      if (!chk(hipMemcpyAsync(A, Ah, (size_t)n * lda * dt_size(ddt), hipMemcpyDeviceToHost, s))) break;
    }
  } while (false);
  (void)hipStreamSynchronize(s);  // the temporaries are in use until the stream drains
  for (void* p : {Bh, Bp, Ap, Ah, (void*)sc})
    if (p) (void)hipFree(p);
  return st;
}

// Allocation-free variant of rbfgs_ridge_hessian for device-resident B and A: the padded FP64
// copy of B, the FP64 output and the two scalars live in the file-scope device array
// `scratch` (one copy per GPU, held until the process ends), cleared by fill kernels rather
// than memsets; nothing is allocated, freed or synchronised.
rbfgs_status rbfgs_ridge_hessian_noalloc(const void* B, int32_t b_dtype, int64_t m, int64_t n, int64_t ldb,
                                         double scale, double lambda, void* A, int32_t a_dtype, int64_t lda,
                                         void* hip_stream) {
  if (!B || !A || m < 1 || n < 1 || n > (1ll << 20) || m > (1ll << 24) || ldb < n || lda < n ||
      (b_dtype != RBFGS_F32 && b_dtype != RBFGS_F64) || (a_dtype != RBFGS_F32 && a_dtype != RBFGS_F64) ||
      !std::isfinite(scale) || !std::isfinite(lambda))
    return RBFGS_E_INVALID_ARG;
  const int64_t np = (n + 127) / 128 * 128, mp = (m + 15) / 16 * 16;
  const size_t b_bytes = align256((size_t)mp * np * sizeof(double)), a_bytes = align256((size_t)np * np * sizeof(double));
  if (b_bytes + a_bytes + 256 > RBFGS_NOALLOC_SCRATCH_BYTES) return RBFGS_E_INVALID_ARG;
  char* base = nullptr;
  if (noalloc_scratch((void**)&base) != hipSuccess) return RBFGS_E_DEVICE;
  hipStream_t s = (hipStream_t)hip_stream;
  double* Bp = (double*)base;
  double* Ap = (double*)(base + b_bytes);
  double* sc = (double*)(base + b_bytes + a_bytes);
  const int sdt = b_dtype == RBFGS_F32 ? DT_F32 : DT_F64, ddt = a_dtype == RBFGS_F32 ? DT_F32 : DT_F64;
  bool ok = fill_f64(Bp, mp * np, 0.0, s) == hipSuccess && fill_f64(Ap, np * np, 0.0, s) == hipSuccess &&
            fill_f64(sc, 1, lambda, s) == hipSuccess && fill_f64(sc + 1, 1, 1.0, s) == hipSuccess &&
            copy_convert(B, sdt, ldb, Bp, DT_F64, np, m, n, s) == hipSuccess &&
            scaled_identity(Ap, np, n, sc, s) == hipSuccess;  // lambda I
  if (ok) {
    GemmArgs g;
    g.M = np; g.N = np; g.K = mp;
    g.A = Bp; g.lda = np; g.a_dt = DT_F64; g.a_kc = false;  // Aop(i, k) = B[k][i]
    g.B = Bp; g.ldb = np; g.b_dt = DT_F64; g.b_kc = false;  // Bop(k, j) = B[k][j]
    g.epi = EPI_SYMUPD; g.C = Ap; g.ldc = np; g.c_dt = DT_F64; g.c2 = scale;
    ok = gemm_f64(g, nullptr, s) == hipSuccess && copy_convert(Ap, DT_F64, np, A, ddt, lda, n, n, s) == hipSuccess;
  }
  return ok ? RBFGS_OK : RBFGS_E_DEVICE;
}

rbfgs_status rbfgs_sketch_coord(uint64_t seed, int64_t k, int64_t n, int32_t q, int32_t* idx_dev, void* hip_stream) {
  if (!idx_dev || n < 1 || q < 1 || q > n || k < 0 || n > (1ll << 20)) return RBFGS_E_INVALID_ARG;
  hipError_t e = sketch_coord(seed, k, n, q, idx_dev, (hipStream_t)hip_stream);
  return e == hipSuccess ? RBFGS_OK : RBFGS_E_DEVICE;
}

}  // extern "C"
