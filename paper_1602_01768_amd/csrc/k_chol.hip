// q x q SPD inverse through Cholesky: G = L L^T, Z = L^-1 (lower) and
// G^-1 = Z^T Z.  G is the sketched matrix S^T A S of eq. (qunac) (its inverse
// enters the update) and of eq. (Cholimprov) (its factor L_G enters the update
// of the inverse factor); the method needs G symmetric positive definite, and
// a non-positive pivot is reported through the status word.
//
// Blocks of order <= 128 run in one workgroup with the whole block in LDS,
// factored in 32-wide panels:
//   F  one wave factors the 32 x 32 diagonal block D = L_pp L_pp^T in registers,
//      half a row per lane;
//   T  the panel below by forward substitution: L_ip = A_ip L_pp^-T, a row per thread;
//   U  trailing update of the lower triangle: A_ik -= L_ip L_kp^T;
// then W_bb = L_bb^-1 for all diagonal blocks at once (a column per thread), and Z
// block row by block row: Z_bb = W_bb, Z_ip = -(W_ii L_i,p:i) Z_p:i,p.
// Larger orders recurse on 2 x 2 blocks with FP64 GEMMs.
#include <math.h>

#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace rb {

namespace {

constexpr int CB = 32;         // panel width
constexpr int LEAF_NT = 512;   // threads of the leaf workgroup
constexpr int LEAF_MAX = 128;  // largest order held in LDS
// the panel (T) and Z-row phases give each thread at most one 4 x 4 micro-tile
static_assert((LEAF_MAX - CB) / 4 * (CB / 4) <= LEAF_NT, "one micro-tile per thread");

// 1 / sqrt(x): hardware estimate refined by two Newton steps (x > 0).
RB_DEV double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Compiler barrier: keeps the loads of an unrolled step from being hoisted into earlier
// steps (which would hold them all in registers at once).
RB_DEV void hold_loads() { __asm__ volatile("" ::: "memory"); }

RB_DEV void lds_fence() {
  // LDS writes of this wave are complete and visible before later LDS reads
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Lower-triangular tile index t -> (ti, tk), ti >= tk, row by row.
RB_DEV void tri_decode(int t, int& ti, int& tk) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  ti = i;
  tk = t - i * (i + 1) / 2;
}

size_t leaf_lds_doubles(int nb) { return (size_t)nb * (nb + 1) + 2 * (size_t)nb + 2 * CB + 1; }

// G: nb x nb block (row-major, ldg), lower triangle read; entries with index >= qv
// are taken as the identity.  Writes Z (row-major, ldz; lower, zero elsewhere and
// on padded indices) and, when Ginv != null, Ginv = Z^T Z (zero on padded indices).
__global__ __launch_bounds__(LEAF_NT) void k_chol_leaf(const double* __restrict__ G, int64_t ldg, int nb, int qv,
                                                       double* __restrict__ Z, int64_t ldz,
                                                       double* __restrict__ Ginv, int64_t ldi, int* status) {
  extern __shared__ double lds[];
  const int P = nb + 1;
  double* a = lds;                  // nb x P: L in the lower triangle, Z^T strictly above it
  double* zd = a + nb * P;          // diag(Z)
  double* dinv = zd + nb;           // 1 / L_jj
  double* colbuf = dinv + nb;       // column j of the diagonal block being factored (x2)
  int* flag = (int*)(colbuf + 2 * CB);
  const int tid = threadIdx.x;

  for (int e = tid; e < nb * nb; e += LEAF_NT) {
    const int i = e / nb, k = e - i * nb;
    if (k > i) continue;
    a[i * P + k] = (i < qv && k < qv) ? G[(int64_t)i * ldg + k] : (i == k ? 1.0 : 0.0);
  }
  if (tid == 0) *flag = 0;
  __syncthreads();

  const int npan = nb / CB;
  for (int pan = 0; pan < npan; ++pan) {
    const int j0 = pan * CB;
    // ---- F: factor the diagonal block D = L_pp L_pp^T in registers.  Lane r + 32h of
    // wave 0 holds columns 16h .. 16h+15 of row r; the sweep is unrolled so every
    // register index is static.
    if (tid < 64) {
      const int r = tid & 31, h = tid >> 5;
      double d[16];
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const int k = 16 * h + kk;
        d[kk] = (k <= r) ? a[(j0 + r) * P + j0 + k] : 0.0;
      }
      bool bad = false;
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int hj = j >> 4, kj = j & 15;
        double* cb = colbuf + (j & 1) * CB;  // two buffers: step j+1 never overwrites what step j reads
        if (h == hj) cb[r] = d[kj];  // column j of the reduced block (rows >= j used)
        lds_fence();
        const double piv = cb[j];
        bad |= !(piv > 0.0);
        const double inv = rsqrt_f64(piv);
        const double lr = (r > j) ? cb[r] * inv : 0.0;  // L[r][j]
        if (h == hj) d[kj] = (r > j) ? lr : (r == j ? piv * inv : d[kj]);
        const double lri = lr * inv;
        if (h == 0) {
#pragma unroll
          for (int k = j + 1; k < 16; ++k) d[k] -= lri * cb[k];  // L[r][j] L[k][j]
        } else {
#pragma unroll
          for (int k = (j + 1 > 16 ? j + 1 : 16); k < CB; ++k) d[k - 16] -= lri * cb[k];
        }
        if (tid == j) dinv[j0 + j] = inv;
      }
      lds_fence();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const int k = 16 * h + kk;
        if (k <= r) a[(j0 + r) * P + j0 + k] = d[kk];
      }
      if (bad) atomicOr(flag, 1);
    }
    __syncthreads();
    if (*flag) {
      if (tid == 0) atomicCAS(status, 0, 3);
      return;
    }
    const int R = nb - j0 - CB;  // rows below the panel
    if (R == 0) break;
    // ---- T: L_ip = A_ip L_pp^-T by forward substitution, one panel row per thread,
    // in place (each thread reads back only what it wrote itself).
    if (tid < R) {
      double* xi = a + (j0 + CB + tid) * P + j0;
      for (int c = 0; c < CB; ++c) {
        const double* lc = a + (j0 + c) * P + j0;
        double s0 = xi[c], s1 = 0.0, s2 = 0.0, s3 = 0.0;  // four chains
        int m = 0;
        for (; m + 4 <= c; m += 4) {
          s0 -= xi[m] * lc[m];
          s1 -= xi[m + 1] * lc[m + 1];
          s2 -= xi[m + 2] * lc[m + 2];
          s3 -= xi[m + 3] * lc[m + 3];
        }
        for (; m < c; ++m) s0 -= xi[m] * lc[m];
        xi[c] = ((s0 + s1) + (s2 + s3)) * dinv[j0 + c];
      }
    }
    __syncthreads();
    // ---- U: trailing update of the lower triangle, 4 x 4 micro-tiles
    {
      const int T4 = R / 4, ntile = T4 * (T4 + 1) / 2, base = j0 + CB;
      for (int t = tid; t < ntile; t += LEAF_NT) {
        int ti, tk;
        tri_decode(t, ti, tk);
        const int i0 = base + 4 * ti, k0 = base + 4 * tk;
        double acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
#pragma unroll 4
        for (int c = 0; c < CB; ++c) {
          double li[4], lk[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            li[x] = a[(i0 + x) * P + j0 + c];
            lk[x] = a[(k0 + x) * P + j0 + c];
          }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] += li[x] * lk[y];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y)
            if (i0 + x >= k0 + y) a[(i0 + x) * P + k0 + y] -= acc[x][y];
      }
      __syncthreads();
    }
  }

  // ---- W_bb = L_bb^-1 for every diagonal block at once, one column c per thread:
  // W[r][c] = (delta_rc - sum_{m < r} L[r][m] W[m][c]) / L[r][r], row by row, written
  // straight to its Z^T slot a[c][r] (r > c) or zd (r = c); each thread reads back
  // only its own column.
  if (tid < nb) {
    const int b0 = (tid / CB) * CB, c = tid % CB;
    double* wc = a + (b0 + c) * P + b0;  // W[m][c] at wc[m] for m > c
    for (int r = c; r < CB; ++r) {
      const double* lr = a + (b0 + r) * P + b0;
      double s0 = (r == c) ? 1.0 : 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;  // four chains
      if (r > c) s0 -= lr[c] * zd[b0 + c];
      int m = c + 1;
      for (; m + 4 <= r; m += 4) {
        s0 -= lr[m] * wc[m];
        s1 -= lr[m + 1] * wc[m + 1];
        s2 -= lr[m + 2] * wc[m + 2];
        s3 -= lr[m + 3] * wc[m + 3];
      }
      for (; m < r; ++m) s0 -= lr[m] * wc[m];
      const double v = ((s0 + s1) + (s2 + s3)) * dinv[b0 + r];
      if (r == c) zd[b0 + c] = v;
      else wc[r] = v;
    }
  }
  __syncthreads();

  // ---- Z off the diagonal blocks, block row by block row; 4 x 4 micro-tiles of the
  // 32 x rb block row, one per thread
  for (int bi = 1; bi < npan; ++bi) {
    const int rb = bi * CB, nt = (CB / 4) * (rb / 4);
    const bool act = tid < nt;
    const int r0 = act ? 4 * (tid % (CB / 4)) : 0, m0 = act ? 4 * (tid / (CB / 4)) : 0;
    // M = W_ii L_i,0:rb (written over L's block row)
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    if (act) {
      double zr[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) zr[x] = zd[rb + r0 + x];
#pragma unroll 4
      for (int q = 0; q < CB; ++q) {
        double wv[4], lv[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int r = r0 + x;
          const double wq = a[(rb + q) * P + rb + r];  // W_ii[r][q] for q < r
          wv[x] = (q < r) ? wq : (q == r ? zr[x] : 0.0);
          lv[x] = a[(rb + q) * P + m0 + x];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] += wv[x] * lv[y];
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) a[(rb + r0 + x) * P + m0 + y] = acc[x][y];
    }
    __syncthreads();
    // Z[rb + r][c] = -sum_{m = c}^{rb - 1} M[r][m] Z[m][c], stored at a[c][rb + r]
    if (act) {
      const int c0 = m0;
      double zc[4];
#pragma unroll
      for (int y = 0; y < 4; ++y) zc[y] = zd[c0 + y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
      // Z[m][c] = 0 for m < c: start at the tile's 32-column block (uniform per wave)
#pragma unroll 4
      for (int m = c0 & ~(CB - 1); m < rb; ++m) {
        double mv[4], zv[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) mv[x] = a[(rb + r0 + x) * P + m];
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int cc = c0 + y;
          const double zm = a[cc * P + m];  // Z[m][cc] for m > cc
          zv[y] = (m > cc) ? zm : (m == cc ? zc[y] : 0.0);
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] += mv[x] * zv[y];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) a[(c0 + y) * P + rb + r0 + x] = -acc[x][y];
    }
    __syncthreads();
  }

  // ---- outputs
  for (int e = tid; e < nb * nb; e += LEAF_NT) {
    const int i = e / nb, k = e - i * nb;
    double v = 0.0;
    if (i < qv && k < qv) v = (k < i) ? a[k * P + i] : (k == i ? zd[i] : 0.0);
    Z[(int64_t)i * ldz + k] = v;
  }
  if (!Ginv) return;
  // Ginv[i][k] = sum_{m >= max(i, k)} Z[m][i] Z[m][k], lower 4 x 4 micro-tiles mirrored
  const int T4 = nb / 4, ntile = T4 * (T4 + 1) / 2;
  for (int t = tid; t < ntile; t += LEAF_NT) {
    int ti, tk;
    tri_decode(t, ti, tk);
    const int i0 = 4 * ti, k0 = 4 * tk;
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    for (int m = i0; m < nb; ++m) {  // Z[m][i] = 0 for m < i, and i0 >= k0
      double zi[4], zk[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int ii = i0 + x, kk = k0 + x;
        zi[x] = (m > ii) ? a[ii * P + m] : (m == ii ? zd[ii] : 0.0);
        zk[x] = (m > kk) ? a[kk * P + m] : (m == kk ? zd[kk] : 0.0);
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += zi[x] * zk[y];
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int i = i0 + x, k = k0 + y;
        if (i < k) continue;
        const double v = (i < qv && k < qv) ? acc[x][y] : 0.0;
        Ginv[(int64_t)i * ldi + k] = v;
        Ginv[(int64_t)k * ldi + i] = v;
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

hipError_t launch_leaf(const double* G, int64_t ldg, int nb, int qv, double* Z, int64_t ldz, double* Ginv,
                       int64_t ldi, int* status, hipStream_t s) {
  static std::once_flag once;  // contexts may be driven from several host threads
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute((const void*)k_chol_leaf, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(leaf_lds_doubles(LEAF_MAX) * sizeof(double)));
  });
  if (attr_err != hipSuccess) return attr_err;
  if (nb % CB || nb > LEAF_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_leaf, dim3(1), dim3(LEAF_NT), leaf_lds_doubles(nb) * sizeof(double), s, G, ldg, nb,
                     qv < 0 ? 0 : (qv > nb ? nb : qv), Z, ldz, Ginv, ldi, status);
  return hipGetLastError();
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
