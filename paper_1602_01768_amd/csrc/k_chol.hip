// q x q SPD inverse through Cholesky: G = L L^T, Z = L^-1 (lower) and
// G^-1 = Z^T Z.  G is the sketched matrix S^T A S of eq. (qunac) (its inverse
// enters the update) and of eq. (Cholimprov) (its factor L_G enters the update
// of the inverse factor); the method needs G symmetric positive definite, and
// a non-positive pivot is reported through the status word.
//
// Blocks of order nb <= 128 run in one workgroup with the whole block in registers
// (4 rows x nb/16 columns per lane, nb/16 waves), by symmetric Gaussian elimination
// applied at once to G and to the identity: step k broadcasts row k through LDS, and
// every row i > k subtracts m_i = G_ki / G_kk times it, the identity part included.
// After nb steps the identity part holds the unit lower factor's inverse L1^-1 (with
// G = L1 D L1^T, the pivots D), so Z = D^-1/2 L1^-1.  Column k of the identity part
// starts at step k, where its entry in row i > k is -m_i; the sweep keeps the entry
// G_ik there instead (= -D_k times it, up to rounding: the broadcast row carries a zero
// in column k), which leaves column k of the identity part scaled by -D_k throughout,
// undone at the end -- so every step is the same multiply-add over all columns, with
// no per-column selection.  One barrier per step, and no phase in which one wave works
// while the others wait.  G^-1 = Z^T Z then runs on the FP64 matrix cores from a copy
// of Z in LDS.  Larger orders recurse on 2 x 2 blocks with FP64 GEMMs.
#include <math.h>

#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace rb {

namespace {

constexpr int CB = 32;         // granule of the block orders
constexpr int LEAF_MAX = 128;  // largest order held in registers

// 1 / sqrt(x): hardware estimate refined by two Newton steps (x > 0).
RB_DEV double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Lower-triangular tile index t -> (ti, tk), ti >= tk, row by row.
RB_DEV void tri_decode(int t, int& ti, int& tk) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  ti = i;
  tk = t - i * (i + 1) / 2;
}

// LDS pitch (doubles) of the copy of Z: rows 16 doubles beyond a multiple of 32 banks
// apart, so that the two rows a half-wave reads in one MFMA operand load use disjoint banks.
template <int NB>
constexpr int zpitch() { return NB + 16; }

typedef double f64x4 __attribute__((ext_vector_type(4)));

// G: nb x nb block (row-major, ldg), lower triangle read; entries with index >= qv are
// taken as the identity.  Writes Z (row-major, ldz; lower, zero elsewhere and on padded
// indices) and, when Ginv != null, Ginv = Z^T Z (zero on padded indices; dynamic LDS of
// nb * zpitch<nb>() doubles).
template <int NB>
__global__ __launch_bounds__(4 * NB) void k_chol_elim(const double* __restrict__ G, int64_t ldg, int qv,
                                                      double* __restrict__ Z, int64_t ldz,
                                                      double* __restrict__ Ginv, int64_t ldi, int* status) {
  constexpr int CPL = NB / 16;  // columns per lane
  constexpr int NW = NB / 16;   // waves: 16 rows each
  constexpr int ZP = zpitch<NB>();
  __shared__ double rowbuf[2][NB];  // row k, double-buffered: one barrier per step
  __shared__ double pinv[NB];       // 1 / D_k
  __shared__ double piv[NB];        // the pivots D
  __shared__ int bad;
  extern __shared__ double zs[];

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rg = lane >> 4, cg = lane & 15;
  const int i0 = 16 * w + 4 * rg, j0 = cg * CPL;  // rows i0 .. i0+3, columns j0 .. j0+CPL-1

  double W[4][CPL];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < CPL; ++y) {
      const int i = i0 + x, j = j0 + y;
      W[x][y] = (i < qv && j < qv) ? G[(int64_t)(i > j ? i : j) * ldg + (i > j ? j : i)] : (i == j ? 1.0 : 0.0);
    }
  if (tid == 0) bad = 0;
  __syncthreads();

  for (int k = 0; k < NB; ++k) {
    double* rb = rowbuf[k & 1];
    // the 16 lanes holding row k publish it (zero in column k), the pivot and its inverse
    if (w == (k >> 4) && rg == ((k >> 2) & 3)) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (x == (k & 3)) {
#pragma unroll
          for (int y = 0; y < CPL; ++y) {
            const bool kk = j0 + y == k;
            rb[j0 + y] = kk ? 0.0 : W[x][y];
            if (kk) {
              piv[k] = W[x][y];
              pinv[k] = 1.0 / W[x][y];
              if (!(W[x][y] > 0.0)) bad = 1;
            }
          }
        }
    }
    __syncthreads();
    if (16 * w + 15 > k) {  // this wave holds rows below k
      const double inv = pinv[k];
      double b[CPL], bi[4];
#pragma unroll
      for (int y = 0; y < CPL; ++y) b[y] = rb[j0 + y];
#pragma unroll
      for (int x = 0; x < 4; ++x) bi[x] = rb[i0 + x];  // G_ki
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const double m = (i0 + x > k) ? bi[x] * inv : 0.0;  // rows <= k are final
#pragma unroll
        for (int y = 0; y < CPL; ++y) W[x][y] = fma(-m, b[y], W[x][y]);
      }
    }
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) atomicCAS(status, 0, 3);
    return;
  }

  // Z = D^-1/2 L1^-1 with L1^-1[i][j] = -W[i][j] / D_j below the diagonal, 1 on it
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int i = i0 + x;
    const double rs = rsqrt_f64(piv[i]);
#pragma unroll
    for (int y = 0; y < CPL; ++y) {
      const int j = j0 + y;
      double v = (j < i) ? -W[x][y] * pinv[j] * rs : (j == i ? rs : 0.0);
      if (i >= qv || j >= qv) v = 0.0;
      Z[(int64_t)i * ldz + j] = v;
      if (Ginv) zs[i * ZP + j] = v;
    }
  }
  if (!Ginv) return;
  __syncthreads();

  // Ginv = Z^T Z on the lower 16 x 16 tiles, mirrored (v_mfma_f64_16x16x4f64: lane l holds
  // A(l%16, l/16), B(l/16, l%16) and the output column l%16, rows l/16 + 4r)
  constexpr int T = NB / 16, NTILE = T * (T + 1) / 2;
  for (int t = w; t < NTILE; t += NW) {
    int ti, tj;
    tri_decode(t, ti, tj);
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int m0 = 16 * ti; m0 < NB; m0 += 4) {  // Z[m][a] = 0 for m < a
      const double av = zs[(m0 + (lane >> 4)) * ZP + 16 * ti + (lane & 15)];
      const double bv = zs[(m0 + (lane >> 4)) * ZP + 16 * tj + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * ti + (lane >> 4) + 4 * r, col = 16 * tj + (lane & 15);
      const double v = (row < qv && col < qv) ? acc[r] : 0.0;
      Ginv[(int64_t)row * ldi + col] = v;
      Ginv[(int64_t)col * ldi + row] = v;
    }
  }
}

__global__ void k_zero_pad_sq(double* M, int64_t ld, int q, int qp) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)qp * qp;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / qp, k = e % qp;
    if (i >= q || k >= q) M[i * ld + k] = 0.0;
  }
}

template <int NB>
hipError_t launch_elim(const double* G, int64_t ldg, int qv, double* Z, int64_t ldz, double* Ginv, int64_t ldi,
                       int* status, hipStream_t s) {
  static std::once_flag once;  // contexts may be driven from several host threads
  static hipError_t attr_err = hipSuccess;
  constexpr size_t zbytes = (size_t)NB * zpitch<NB>() * sizeof(double);
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute((const void*)k_chol_elim<NB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)zbytes);
  });
  if (attr_err != hipSuccess) return attr_err;
  hipLaunchKernelGGL(k_chol_elim<NB>, dim3(1), dim3(4 * NB), Ginv ? zbytes : 0, s, G, ldg, qv, Z, ldz, Ginv, ldi,
                     status);
  return hipGetLastError();
}

hipError_t launch_leaf(const double* G, int64_t ldg, int nb, int qv, double* Z, int64_t ldz, double* Ginv,
                       int64_t ldi, int* status, hipStream_t s) {
  qv = qv < 0 ? 0 : (qv > nb ? nb : qv);
  switch (nb) {
    case 32: return launch_elim<32>(G, ldg, qv, Z, ldz, Ginv, ldi, status, s);
    case 64: return launch_elim<64>(G, ldg, qv, Z, ldz, Ginv, ldi, status, s);
    case 96: return launch_elim<96>(G, ldg, qv, Z, ldz, Ginv, ldi, status, s);
    case 128: return launch_elim<128>(G, ldg, qv, Z, ldz, Ginv, ldi, status, s);
    default: return hipErrorInvalidValue;
  }
}

// Recursive 2 x 2 block inverse-Cholesky on a padded block of order `size`:
//   Z11 = chol(G11)^-1;  L21 = G21 Z11^T;  G22' = G22 - L21 L21^T;  Z22 = chol(G22')^-1;
//   Z21 = -Z22 L21 Z11.   (Z = L^-1 with L = [[L11, 0], [L21, L22]].)
hipError_t chol_rec(const double* G, int64_t ldg, int size, int qv, double* Z, int64_t ldz, double* work,
                    int* status, hipStream_t s) {
  if (size <= LEAF_MAX) return launch_leaf(G, ldg, size, qv, Z, ldz, nullptr, 0, status, s);
  const int s1 = ((size / 2 + CB - 1) / CB) * CB, s2 = size - s1;
  hipError_t e;
  if ((e = chol_rec(G, ldg, s1, qv, Z, ldz, work, status, s)) != hipSuccess) return e;
  double* L21 = work;                    // s2 x s1 row-major
  double* G22 = L21 + (int64_t)s2 * s1;  // s2 x s2
  double* T = G22 + (int64_t)s2 * s2;    // s2 x s1
  double* next = T + (int64_t)s2 * s1;
  // L21 = G21 Z11^T : Aop(m,k) = G21[m][k], Bop(k,n) = Z11[n][k]  (padded rows of G are zero)
  GemmArgs g;
  g.M = s2; g.N = s1; g.K = s1;
  g.A = G + (int64_t)s1 * ldg; g.lda = ldg; g.a_kc = true;
  g.B = Z; g.ldb = ldz; g.b_kc = true;
  g.epi = EPI_ROWSTORE; g.C = L21; g.ldc = s1; g.c2 = 1.0;
  if ((e = gemm_f64(g, nullptr, s)) != hipSuccess) return e;
  // G22' = G22 - L21 L21^T (symmetric, so the column-major store is the row-major one)
  GemmArgs h;
  h.M = s2; h.N = s2; h.K = s1;
  h.A = L21; h.lda = s1; h.a_kc = true;
  h.B = L21; h.ldb = s1; h.b_kc = true;
  h.epi = EPI_COLSTORE; h.C = G22; h.ldc = s2; h.c2 = -1.0;
  h.B0 = G + (int64_t)s1 * ldg + s1; h.ld01 = ldg; h.c0 = 1.0;
  if ((e = gemm_f64(h, nullptr, s)) != hipSuccess) return e;
  if ((e = chol_rec(G22, s2, s2, qv - s1, Z + (int64_t)s1 * ldz + s1, ldz, next, status, s)) != hipSuccess)
    return e;
  // T = L21 Z11
  GemmArgs t;
  t.M = s2; t.N = s1; t.K = s1;
  t.A = L21; t.lda = s1; t.a_kc = true;
  t.B = Z; t.ldb = ldz; t.b_kc = false;
  t.epi = EPI_ROWSTORE; t.C = T; t.ldc = s1; t.c2 = 1.0;
  if ((e = gemm_f64(t, nullptr, s)) != hipSuccess) return e;
  // Z21 = -Z22 T
  GemmArgs z;
  z.M = s2; z.N = s1; z.K = s2;
  z.A = Z + (int64_t)s1 * ldz + s1; z.lda = ldz; z.a_kc = true;
  z.B = T; z.ldb = s1; z.b_kc = false;
  z.epi = EPI_ROWSTORE; z.C = Z + (int64_t)s1 * ldz; z.ldc = ldz; z.c2 = -1.0;
  return gemm_f64(z, nullptr, s);
}

}  // namespace

size_t chol_inv_work_doubles(int q) {
  const int64_t qp = ((int64_t)q + 31) / 32 * 32;
  return (size_t)(4 * qp * qp + 1024);
}

hipError_t chol_inv(const double* G, int64_t ldg, int q, double* Z, double* Ginv, int64_t ld, double* work,
                    int* status, hipStream_t s) {
  const int qp = (q + CB - 1) / CB * CB;
  if (qp <= LEAF_MAX) return launch_leaf(G, ldg, qp, q, Z, ld, Ginv, ld, status, s);
  hipError_t e = chol_rec(G, ldg, qp, q, Z, ld, work, status, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_pad_sq, dim3(64), dim3(256), 0, s, Z, ld, q, qp);
  if (!Ginv) return hipGetLastError();
  // Ginv = Z^T Z : Aop(i,k) = Z[k][i], Bop(k,j) = Z[k][j]
  GemmArgs g;
  g.M = qp; g.N = qp; g.K = qp;
  g.A = Z; g.lda = ld; g.a_kc = false;
  g.B = Z; g.ldb = ld; g.b_kc = false;
  g.epi = EPI_ROWSTORE; g.C = Ginv; g.ldc = ld; g.c2 = 1.0;
  return gemm_f64(g, nullptr, s);
}

}  // namespace rb
