// Launchers of the RBFGS HIP kernels (host side).  Every matrix handled here is
// zero-padded: the matrix order n to np (a multiple of 256), the sketch size q to
// qp (a multiple of 32), and every pad entry of every operand is zero, so tiles
// never need bounds checks and pad entries stay zero through every product.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rb {

enum DType : int { DT_F32 = 0, DT_F64 = 1, DT_BF16 = 2 };

// ------------------------------------------------------------- FP64 MFMA GEMM
// C = sum_k Aop(m,k) Bop(k,n) over m < M, n < N, k < K (all multiples of the tile).
//   Aop(m,k) = A[m*lda + k] (a_kc) or A[k*lda + m]
//   Bop(k,n) = B[n*ldb + k] (b_kc) or B[k*ldb + n]
// Inputs of type F32/F64/BF16 are converted to FP64; accumulation is FP64 MFMA.
enum Epi : int {
  EPI_PARTIAL = 0,  // split-K partial sums, double, [split][n*M + m] (reduce_partials finishes)
  EPI_COLSTORE = 1, // C[m + n*ldc] = c2*acc + c0*B0[m + n*ld01] + c1*B1[m + n*ld01]
  EPI_SYMUPD = 2,   // X += c2*acc on lower tiles, mirrored to keep X exactly symmetric
  EPI_ADDROW = 3,   // C[m*ldc + n] += c2*acc
  EPI_RESID = 4,    // red[block] = sum over m,n < nvalid of (delta_mn - acc)^2
  EPI_ROWSTORE = 5  // C[m*ldc + n] = c2*acc
};

struct GemmArgs {
  int64_t M = 0, N = 0, K = 0;
  const void* A = nullptr; int64_t lda = 0; int a_dt = DT_F64; bool a_kc = true;
  const void* B = nullptr; int64_t ldb = 0; int b_dt = DT_F64; bool b_kc = true;
  int splitk = 1;
  int epi = EPI_COLSTORE;
  void* C = nullptr; int64_t ldc = 0; int c_dt = DT_F64;
  const void* B0 = nullptr; int b0_dt = DT_F64;
  const void* B1 = nullptr; int b1_dt = DT_F64;
  int64_t ld01 = 0;
  double c0 = 0, c1 = 0, c2 = 1;
  double* red = nullptr;
  int64_t nvalid = 0;
  // bf16 GEMM only: plane strides of pre-split operands, split counts
  int64_t a_plane = 0, b_plane = 0;
  // square products (EPI_SYMUPD, EPI_ADDROW): optional tile order (tile row, tile column),
  // handed out so that each XCD (blockIdx % 8) takes a contiguous run of it
  const int2* tiles = nullptr;
  int64_t ntiles = 0;
  // optional event recorded on the stream between the product kernel and its split-K
  // reduction (timing of the product kernel alone)
  hipEvent_t mark = nullptr;
  // bf16 split-K reduction only: when est_red is set, the reduction also writes, per
  // workgroup, the sum of (est_S - C)^2 over its part of C (est_S: bf16, column-major
  // with leading dimension ldc) to est_red[workgroup]; reduce_blocks_f32 gives the count
  const __bf16* est_S = nullptr;
  double* est_red = nullptr;
  // bf16 tall-skinny products: tile width along N (0: the widest of 256/128/64/32 dividing N)
  int bn = 0;
  // bf16 symmetric update (EPI_SYMUPD): write the lower tiles only, no mirrored copies
  bool lower_only = false;
  // streamed product: the bf16 planes of B are tile-major (see split_planes; ldb = the number
  // of columns of B the planes hold)
  bool b_tiled = false;
  // bf16 square update: bf16 pieces per operand (2, or 3 for the symmetric update)
  int upd_pieces = 2;
};

// Tile order for an n x n product of T x T tiles: super-tiles of S x S tiles in row-major
// order, tiles row-major inside each; lower triangle only when `lower`.  Returns the count.
int64_t make_tile_order(int T, int S, bool lower, int2* out);

hipError_t gemm_f64(const GemmArgs& g, void* partial_ws, hipStream_t s);
// Sum split-K partials ([split][M*N] double, column-major M x N) into the
// COLSTORE epilogue of g (which may read B0/B1).
hipError_t reduce_partials_f64(const GemmArgs& g, const double* partial, hipStream_t s);
int64_t gemm_f64_blocks(const GemmArgs& g);

// ------------------------------------------------------------ bf16 MFMA GEMM
// Operand kinds for the mixed-precision GEMM.
enum OpKind : int {
  OK_F32_KC = 0,    // FP32, contiguous along k, split into bf16 pieces on load
  OK_F32_MC = 1,    // FP32, contiguous along m (or n), split on load
  OK_BF16_KC = 2,   // pre-split bf16 planes, contiguous along k (plane p at base + p*plane)
  OK_BF16_MC = 3,   // one bf16 plane, contiguous along m (or n)
  OK_F32_SYM = 4    // FP32 symmetric, current on its lower 128 x 128 tiles only (streamed product)
};
struct MixedGemm {
  // the products write FP32 unless g.c_dt is set to DT_F64 explicitly (q x q results)
  MixedGemm() { g.c_dt = DT_F32; }
  GemmArgs g;
  int a_kind = OK_F32_KC, b_kind = OK_F32_KC;
  int na = 2, nb = 2;   // pieces per operand
  int pmax = 1;         // passes: all piece pairs (i, j) with i + j <= pmax
};
hipError_t gemm_bf16(const MixedGemm& mg, void* partial_ws, hipStream_t s);
// Streamed tall-skinny product (k_tall.hip): A FP32 k-contiguous or transposed (na pieces), B bf16 planes
// (nb pieces, k-contiguous rows), N a multiple of 128, M a multiple of 32 and >= 1024, split-K
// dividing 8.  gemm_bf16 takes it for every product it supports.
bool tall_stream_supported(const MixedGemm& mg);
hipError_t tall_stream(const GemmArgs& run, const MixedGemm& mg, hipStream_t s);
// bf16 planes of a column-major n x q panel (leading dimension ldi), tile-major for the streamed
// product: bf16 piece p of in[j * ldi + i] goes to out[p * rows * cols + (i / 32) * 32 cols +
// j * 32 + i % 32], so that the 32-deep k tile of every column is one contiguous block.  np = 1
// copies a bf16 panel, 2 or 3 split an FP32 one (rows a multiple of 32).
hipError_t split_planes(const void* in, int64_t rows, int64_t cols, int64_t ldi, int np, __bf16* out, hipStream_t s);
// Tile edge of the bf16 square products (EPI_SYMUPD / EPI_ADDROW) for order M and depth K.
int bf16_square_tile(int64_t M, int64_t K, int epi);
// Sum the FP32 split-K partials of a bf16 product (COLSTORE epilogue of g): C = c2 * sum
// + c0 * B0 (FP32) + c1 * B1 (FP32 or bf16, b1_dt), column-major; C is FP32 or FP64 (c_dt).
hipError_t reduce_partials_f32(const GemmArgs& g, const float* partial, hipStream_t s);
// Square update with operands loaded straight into LDS, 2 x 2 bf16 pieces: EPI_SYMUPD
// (lower tiles, mirrored) or EPI_ADDROW (every tile); blocks as gemm_bf16_blocks gives
// for 128 x 128 tiles.
hipError_t symupd_bf16_dma(const GemmArgs& g, int64_t blocks, hipStream_t s);
// Copy the strictly lower 128 x 128 tiles of the FP32 n x n matrix X (T tiles a side) onto
// the upper ones, transposed: X held on its lower tiles becomes whole again.
hipError_t mirror_lower(float* X, int64_t ld, int64_t T, hipStream_t s);
int64_t reduce_blocks_f32(const GemmArgs& g);
int64_t gemm_bf16_blocks(const MixedGemm& mg);

// Pack an FP32 column-major panel (rows x cols, ld_in) into bf16 hi/lo planes of ld_out columns,
// starting at column col_off: row-major (tile = 0), or tile-major for the symmetric update
// (tile rows per row tile, and within one the 32-column stages one after another, each
// tile x 32 row-major: entry (r, c) at (r / tile) tile ld_out + (c / 32) 32 tile +
// (r % tile) 32 + c % 32).  With mid given, three pieces: hi, mid and lo.
hipError_t pack_split2(const float* in, int64_t ld_in, int64_t rows, int64_t cols,
                       __bf16* hi, __bf16* lo, int64_t ld_out, int64_t col_off, hipStream_t s, int64_t tile = 0,
                       __bf16* mid = nullptr);

// ------------------------------------------------------------------ sketches
hipError_t sketch_gauss(uint64_t seed, int64_t k, int64_t n, int32_t q, void* S, int dt, int64_t ld, hipStream_t s,
                        const int64_t* kbase = nullptr);  // iteration k (+ *kbase when given)
// *c += v (one thread; a kernel so that it can sit in a captured graph)
hipError_t add_i64(int64_t* c, int64_t v, hipStream_t s);
hipError_t sketch_coord(uint64_t seed, int64_t k, int64_t n, int32_t q, int32_t* idx,
                        hipStream_t s);

// ------------------------------------------------------------ small kernels
// q x q SPD inverse through Cholesky: Z = L^-1 (lower) and Ginv = Z^T Z, both
// qp x qp row-major with zero pad; *status set to 3 on a pivot <= 0 or NaN.
// q <= 128 runs in one workgroup; larger q recurses on 2 x 2 blocks with FP64 GEMMs.
hipError_t chol_inv(const double* G, int64_t ldg, int q, double* Z, double* Ginv,
                    int64_t ld, double* work, int* status, hipStream_t s);
size_t chol_inv_work_doubles(int q);

// Y[i + j*ldy] = A[C_j*lda + i] (A symmetric), G[a*ldg + b] = A[C_a*lda + C_b].
hipError_t gather_cols_sym(const void* A, int a_dt, int64_t lda, const int32_t* C, int q,
                           int64_t np, void* Y, int y_dt, int64_t ldy, double* G, int64_t ldg,
                           hipStream_t s);
// S[i + j*lds] = L[i*ldl + C_j] (general L).
hipError_t gather_cols_gen(const void* L, int l_dt, int64_t ldl, const int32_t* C, int q,
                           int64_t np, void* S, int s_dt, int64_t lds, hipStream_t s);
// sum (Sk - V)^2 over the n x q block, Sk dense (sk_dt) or coordinate (C != null).
// Writes est = sum * scale (* dscale[0] when given) to est[0] and adds it to est[2] (the
// window sum the stopping test reads); sets *status = 4 when not finite.
hipError_t estimator(const void* Sk, int sk_dt, const int32_t* C, const void* V, int v_dt,
                     int64_t ld, int64_t n, int q, double scale, double* red, double* est,
                     int* status, hipStream_t s, const double* dscale = nullptr);
// Deterministic sum of `count` doubles into *out (single workgroup).
hipError_t reduce_sum(const double* in, int64_t count, double* out, hipStream_t s);
// out[0] = scale * sum of `count` doubles, also added to out[2] (an estimate's window sum);
// *status = 4 when the sum is not finite.
hipError_t reduce_sum_scaled(const double* in, int64_t count, double* out, double scale, int* status,
                             hipStream_t s);
// rows C_a of W' (col-major, ld): W'[C_a + b*ld] -= 0.5*(a==b) + 0.5*GH[a*ldgh + b]
hipError_t coord_wprime_fix(void* W, int w_dt, int64_t ld, const int32_t* C, int q,
                            const double* GH, int64_t ldgh, hipStream_t s);
// rows C_a of Q^T (col-major): Qt[C_a + b*ld] += M[a*ldm + b]
hipError_t coord_add_rows(void* Qt, int dt, int64_t ld, const int32_t* C, int q,
                          const double* M, int64_t ldm, hipStream_t s);
// Fixed-sketch coordinate update of symmetric X given R = Ginv W'^T (q x np, row-major):
// rows C_a: X[C_a, j] -= R[a, j] + (j = C_b ? R[b, C_a] : 0), then columns mirrored.
hipError_t coord_sym_update(void* X, int x_dt, int64_t ldx, const int32_t* C, int32_t* pos,
                            int q, int64_t np, const void* R, int r_dt, int64_t ldr, hipStream_t s);
// X = I on the leading n x n block of the np x np zero matrix.
hipError_t set_identity(void* X, int dt, int64_t ld, int64_t n, hipStream_t s);
// Copy (with conversion) an n x n row-major matrix between element types.
hipError_t copy_convert(const void* src, int s_dt, int64_t lds, void* dst, int d_dt, int64_t ldd,
                        int64_t rows, int64_t cols, hipStream_t s);
// 1 if any of the n x n entries is non-finite or (sym) A[i][j] != A[j][i] (exact), accumulated into *flag.
hipError_t check_sym_finite(const void* A, int dt, int64_t lda, int64_t n, int* flag, hipStream_t s, bool sym = true);
// out = a X + b Y on column-major rows x cols panels (leading dimension ld), any element types.
hipError_t panel_axpby(const void* X, int xdt, double a, const void* Y, int ydt, double b, void* out, int odt,
                       int64_t rows, int64_t cols, int64_t ld, hipStream_t s);
// Transposed copy with conversion: dst[j*ldd + i] = src[i*lds + j], i < rows, j < cols.
hipError_t copy_transpose(const void* src, int s_dt, int64_t lds, void* dst, int d_dt, int64_t ldd, int64_t rows,
                          int64_t cols, hipStream_t s);
// Comparison methods (Newton-Schulz, MR), n x n row-major FP64 with leading dimension ld.
// sigma ~ ||A||_2 by `steps` power-method steps from the all-ones vector (v, w: n doubles).
hipError_t power_norm(const double* A, int64_t ld, int64_t n, int steps, double* v, double* w, double* sigma,
                      hipStream_t s);
// X = 0.99 A^T / sigma^2 on the n x n block.
hipError_t ns_start(const double* A, int64_t ld, int64_t n, const double* sigma, double* X, hipStream_t s);
// Per-block partial sums (sums_blocks(n) blocks): mode 0 sum (I - T)^2; 1 T := I - T and sum T^2;
// 2 pairs (sum T Q, sum Q^2); 3 pairs (trace T, sum T^2).
int sums_blocks(int64_t n);
hipError_t mat_sums(double* T, const double* Q, int64_t ld, int64_t n, int mode, double* red, hipStream_t s);
hipError_t reduce_pairs(const double* red, int nb, double* out, hipStream_t s);
// X += (sc[0] / sc[1]) P over `total` entries; X = (sc[0] / sc[1]) I on the n x n block.
hipError_t axpy_ratio(double* X, const double* P, int64_t total, const double* sc, hipStream_t s);
hipError_t scaled_identity(double* X, int64_t ld, int64_t n, const double* sc, hipStream_t s);
// v[0 .. count) = x (a kernel, so that it may be captured into a graph)
hipError_t fill_f64(double* v, int64_t count, double x, hipStream_t s);
// Conjugate gradients: y = M v (transpose: M^T v) for an n x n row-major M (FP32/FP64,
// ld % 4 == 0), FP64 vectors; `part` holds GEMV_T_CHUNKS * n doubles for the transpose.
constexpr int GEMV_T_CHUNKS = 32;
hipError_t gemv(const void* M, int dt, int64_t ld, int64_t n, bool transpose, const double* v, double* y,
                double* part, hipStream_t s);
hipError_t dot(const double* a, const double* b, int64_t n, double* out, hipStream_t s);
// x += (sc[num]/sc[den]) p, r -= (sc[num]/sc[den]) Ap;  p = z + (sc[num]/sc[den]) p.
hipError_t cg_xr(double* x, double* r, const double* p, const double* Ap, int64_t n, const double* sc, int num, int den,
                 hipStream_t s);
hipError_t cg_p(double* p, const double* z, int64_t n, const double* sc, int num, int den, hipStream_t s);
// Dense ld x qp column-major coordinate sketch from the indices C (q of them): ones at (C_j, j).
hipError_t coord_dense(const int32_t* C, int q, void* S, int dt, int64_t ld, int64_t qp, hipStream_t s);


// ---- partition sampling (eq. ihsih0 over consecutive blocks of q; q divides n)
// Draw block i of [0, n/q) with probability w_i / sum w, w_i = max(0, sum_{j in C_i} t_j),
// from word 0 of iteration k's stream (kind 3); idx[0..q) = C_i; ht = 1/p_i (optional).
hipError_t sample_partition(const double* t, int64_t n, int32_t q, uint64_t seed, int64_t k, int32_t* idx, double* ht,
                            int* status, hipStream_t s);
// t_j = A_jj (FP64), j < n.
hipError_t diag_weights(const void* A, int dt, int64_t ld, int64_t n, double* t, hipStream_t s);
// t_j += sum_c V_jc W_jc + [C[0] <= j < C[0] + q]  (AdaRBFGS: V = L^T Y, W = -L^T Y G^-1).
hipError_t part_weights(const void* V, const void* W, int dt, int64_t ld, int64_t n, int q, const int32_t* C, double* t,
                        hipStream_t s);
// t[C[c]] = sum_r P_rc Q_rc, c < q (column-major n x q panels).
hipError_t col_dots(const void* P, const void* Q, int dt, int64_t ld, int64_t n, int q, const int32_t* C, double* t,
                    hipStream_t s);
// idx[c] = start + c, c < q.
hipError_t fill_block(int32_t* idx, int64_t start, int q, hipStream_t s);

}  // namespace rb
