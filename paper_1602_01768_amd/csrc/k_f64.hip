// FP64 kernels: tiled FP64-MFMA GEMM with epilogues, the q x q Cholesky-based
// inverse, gathers, the per-step estimator and small elementwise kernels.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace rb {

RB_DEV double load_any(const void* p, int dt, int64_t i) {
  if (dt == DT_F32) return (double)((const float*)p)[i];
  if (dt == DT_BF16) return (double)(float)((const __bf16*)p)[i];
  return ((const double*)p)[i];
}
RB_DEV void store_any(void* p, int dt, int64_t i, double v) {
  if (dt == DT_F32) ((float*)p)[i] = (float)v;
  else if (dt == DT_BF16) ((__bf16*)p)[i] = (__bf16)(float)v;
  else ((double*)p)[i] = v;
}
RB_DEV double round_to(int dt, double v) { return dt == DT_F32 ? (double)(float)v : v; }

// Lower-triangular tile index t -> (ti, tj), ti >= tj, row by row.
RB_DEV void tri_index(int64_t t, int64_t& ti, int64_t& tj) {
  int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// Block-wide sum of one double per thread (blockDim = 256); result valid in thread 0.
RB_DEV double block_sum_256(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return s;
}

// ------------------------------------------------------------------ GEMM
#ifndef GEMV_T_COLS
#define GEMV_T_COLS 2  // columns per thread of the transposed product y = M^T v (CG); 1, 2, 4 measured: 2
#endif
#ifndef GEMV_RPW
#define GEMV_RPW 2  // rows per wave of the row product y = M v (CG); 1, 2, 4, 8 measured: 2 fastest
#endif
// 256 threads, 4 waves as 2 x 2; wave tile (BM/2) x (BN/2) of 16 x 16 MFMA blocks
// (v_mfma_f64_16x16x4f64: lane l holds A(l%16, l/16), B(l/16, l%16) and the
// output column l%16, rows l/16 + 4r).  BK = 16 staged through LDS with a
// one-tile register prefetch.
// 128 x 128 tiles hold 64 FP64 accumulators per lane and run one wave per SIMD;
// smaller tiles ask for two.
template <int BM, int BN, bool AKC, bool BKC, int EPI>
__global__ __launch_bounds__(256, (BM * BN >= 128 * 128) ? 1 : 2) void k_gemm_f64(GemmArgs g) {
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  constexpr int AP = BM * BK / 256, BP = BN * BK / 256;
  constexpr int LOOP_D = BK * (BM + 1) + BK * (BN + 1);
  constexpr int EPI_D = 4 * 16 * (WM + 1);
  constexpr int SM = LOOP_D > EPI_D ? LOOP_D : EPI_D;
  __shared__ double smem[SM];
  double* As = smem;
  double* Bs = smem + BK * (BM + 1);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t MT = g.M / BM;
  int64_t mt, nt;
  int kc = 0;
  bool diag = false;
  const int64_t bid = blockIdx.x;
  if constexpr (EPI == EPI_SYMUPD || EPI == EPI_ADDROW) {
    // square products: each XCD (blockIdx % 8) takes a contiguous run of the tile order
    const int64_t T = g.M / BM;
    const int64_t NTT = g.tiles ? g.ntiles : (EPI == EPI_SYMUPD ? T * (T + 1) / 2 : T * T);
    const int64_t per = (NTT + 7) / 8, t = (bid % 8) * per + bid / 8;
    if (t >= NTT) return;
    if (g.tiles) {
      mt = g.tiles[t].x;
      nt = g.tiles[t].y;
    } else if (EPI == EPI_SYMUPD) {
      tri_index(t, mt, nt);
    } else {
      mt = t / T;
      nt = t % T;
    }
    diag = (EPI == EPI_SYMUPD) && (mt == nt);
  } else {
    kc = (int)(bid % g.splitk);
    const int64_t r = bid / g.splitk;
    mt = r % MT;
    nt = r / MT;
  }
  const int64_t kchunk = g.K / g.splitk;
  const int64_t kbeg = kc * kchunk, kend = kbeg + kchunk;
  const int64_t m0 = mt * BM, n0 = nt * BN;

  double ra[AP], rbv[BP];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < AP; ++i) {
      const int e = tid + 256 * i;
      int mm, kk;
      if (AKC) { mm = e / BK; kk = e % BK; ra[i] = load_any(g.A, g.a_dt, (m0 + mm) * g.lda + k0 + kk); }
      else { kk = e / BM; mm = e % BM; ra[i] = load_any(g.A, g.a_dt, (k0 + kk) * g.lda + m0 + mm); }
    }
#pragma unroll
    for (int i = 0; i < BP; ++i) {
      const int e = tid + 256 * i;
      int nn, kk;
      if (BKC) { nn = e / BK; kk = e % BK; rbv[i] = load_any(g.B, g.b_dt, (n0 + nn) * g.ldb + k0 + kk); }
      else { kk = e / BN; nn = e % BN; rbv[i] = load_any(g.B, g.b_dt, (k0 + kk) * g.ldb + n0 + nn); }
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int i = 0; i < AP; ++i) {
      const int e = tid + 256 * i;
      const int mm = AKC ? e / BK : e % BM, kk = AKC ? e % BK : e / BM;
      As[kk * (BM + 1) + mm] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BP; ++i) {
      const int e = tid + 256 * i;
      const int nn = BKC ? e / BK : e % BN, kk = BKC ? e % BK : e / BN;
      Bs[kk * (BN + 1) + nn] = rbv[i];
    }
  };

  f64x4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};

  gload(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + BK < kend) gload(k0 + BK);
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      double av[FM], bv[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) av[a] = As[kr * (BM + 1) + wm * WM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < FN; ++b) bv[b] = Bs[kr * (BN + 1) + wn * WN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }

  // ---------------------------------------------------------------- epilogue
  const int lr = lane >> 4, lc = lane & 15;
  if constexpr (EPI == EPI_RESID) {
    double s = 0;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + wm * WM + a * 16 + lr + 4 * r, n = n0 + wn * WN + b * 16 + lc;
          if (m < g.nvalid && n < g.nvalid) {
            const double d = (m == n ? 1.0 : 0.0) - acc[a][b][r];
            s += d * d;
          }
        }
    __syncthreads();
    const double t = block_sum_256(s, smem);
    if (tid == 0) g.red[bid] = t;
    return;
  }
  if constexpr (EPI == EPI_SYMUPD) {
    __syncthreads();
    double* R = smem + wave * 16 * (WM + 1);
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      const int64_t nb = n0 + wn * WN + b * 16;
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ml = a * 16 + lr + 4 * r;
          const int64_t m = m0 + wm * WM + ml, n = nb + lc;
          const int64_t idx = m * g.ldc + n;
          const double nv = round_to(g.c_dt, load_any(g.C, g.c_dt, idx) + g.c2 * acc[a][b][r]);
          if (!diag || m >= n) store_any(g.C, g.c_dt, idx, nv);
          R[lc * (WM + 1) + ml] = nv;
        }
      __syncthreads();
      if (lane < WM) {
        const int64_t mrow = m0 + wm * WM + lane;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int64_t ncol = nb + c;
          if (!diag || mrow > ncol) store_any(g.C, g.c_dt, ncol * g.ldc + mrow, R[c * (WM + 1) + lane]);
        }
      }
      __syncthreads();
    }
    return;
  }
  // element (a, b, r) of the wave tile: row a*16 + lr + 4r, column b*16 + lc
  const int64_t wm0 = m0 + wm * WM, wn0 = n0 + wn * WN;
  if constexpr (EPI == EPI_PARTIAL) {
    double* P = (double*)g.C + (int64_t)kc * g.M * g.N + wn0 * g.M + wm0;
    const int ldp = (int)g.M;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) P[(b * 16 + lc) * ldp + a * 16 + lr + 4 * r] = acc[a][b][r];
  } else if constexpr (EPI == EPI_COLSTORE) {
    const int ldc = (int)g.ldc, ld01 = (int)g.ld01;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = wm0 + a * 16 + lr + 4 * r, n = wn0 + b * 16 + lc;
          double o = g.c2 * acc[a][b][r];
          if (g.B0) o += g.c0 * load_any(g.B0, g.b0_dt, m + n * ld01);
          if (g.B1) o += g.c1 * load_any(g.B1, g.b1_dt, m + n * ld01);
          store_any(g.C, g.c_dt, m + n * ldc, o);
        }
  } else {  // EPI_ADDROW, EPI_ROWSTORE
    const int ldc = (int)g.ldc;
    const int64_t base = wm0 * g.ldc + wn0;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t idx = base + (a * 16 + lr + 4 * r) * ldc + b * 16 + lc;
          if constexpr (EPI == EPI_ADDROW) store_any(g.C, g.c_dt, idx, load_any(g.C, g.c_dt, idx) + g.c2 * acc[a][b][r]);
          else store_any(g.C, g.c_dt, idx, g.c2 * acc[a][b][r]);
        }
  }
}

// C[m + n*ldc] = c2 * sum_k P[k][n*M + m] (+ c0 B0 + c1 B1); grid (M / 256, N).
__global__ void k_reduce_partials_f64(GemmArgs g, const double* P) {
  const int64_t n = blockIdx.y, m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= g.M) return;
  const int64_t MN = g.M * g.N, o = n * g.M + m;
  double s = 0;
  for (int k = 0; k < g.splitk; ++k) s += P[(int64_t)k * MN + o];
  double v = g.c2 * s;
  if (g.B0) v += g.c0 * load_any(g.B0, g.b0_dt, m + n * g.ld01);
  if (g.B1) v += g.c1 * load_any(g.B1, g.b1_dt, m + n * g.ld01);
  store_any(g.C, g.c_dt, m + n * g.ldc, v);
}

// Tile shape of the column/row-store products: the largest tile that still gives
// enough workgroups (M, N multiples of 32).
static void pick_tiles(const GemmArgs& g, int& BM, int& BN) {
  const int64_t sk = g.splitk;
  if (g.M % 128 == 0 && g.N % 128 == 0 && (g.M / 128) * (g.N / 128) * sk >= 256) { BM = BN = 128; return; }
  if (g.M % 64 == 0 && g.N % 64 == 0 && (g.M / 64) * (g.N / 64) * sk >= 64) { BM = BN = 64; return; }
  if (g.M % 128 == 0 && (g.M / 128) * (g.N / 32) * sk >= 256) { BM = 128; BN = 32; return; }
  if (g.N % 128 == 0 && (g.M / 32) * (g.N / 128) * sk >= 256) { BM = 32; BN = 128; return; }
  BM = BN = 32;
}

int64_t gemm_f64_blocks(const GemmArgs& g) {
  if (g.epi == EPI_SYMUPD || g.epi == EPI_ADDROW || g.epi == EPI_RESID) {
    const int64_t T = g.M / 128;
    if (g.epi == EPI_RESID) return T * (g.N / 128);
    const int64_t NTT = g.tiles ? g.ntiles : (g.epi == EPI_SYMUPD ? T * (T + 1) / 2 : T * T);
    return (NTT + 7) / 8 * 8;
  }
  int BM, BN;
  pick_tiles(g, BM, BN);
  return (g.M / BM) * (g.N / BN) * g.splitk;
}

template <int BM, int BN, int EPI>
static void launch_f64(const GemmArgs& g, int64_t blocks, hipStream_t s) {
  if (g.a_kc && g.b_kc) hipLaunchKernelGGL((k_gemm_f64<BM, BN, true, true, EPI>), dim3(blocks), dim3(256), 0, s, g);
  else if (g.a_kc) hipLaunchKernelGGL((k_gemm_f64<BM, BN, true, false, EPI>), dim3(blocks), dim3(256), 0, s, g);
  else if (g.b_kc) hipLaunchKernelGGL((k_gemm_f64<BM, BN, false, true, EPI>), dim3(blocks), dim3(256), 0, s, g);
  else hipLaunchKernelGGL((k_gemm_f64<BM, BN, false, false, EPI>), dim3(blocks), dim3(256), 0, s, g);
}

template <int BM, int BN>
static hipError_t launch_f64_epi(const GemmArgs& g, int64_t blocks, hipStream_t s) {
  switch (g.epi) {
    case EPI_PARTIAL: launch_f64<BM, BN, EPI_PARTIAL>(g, blocks, s); break;
    case EPI_COLSTORE: launch_f64<BM, BN, EPI_COLSTORE>(g, blocks, s); break;
    case EPI_ROWSTORE: launch_f64<BM, BN, EPI_ROWSTORE>(g, blocks, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

hipError_t gemm_f64(const GemmArgs& gin, void* partial_ws, hipStream_t s) {
  GemmArgs g = gin;
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
  if (g.M % 32 || g.N % 32 || g.K % 16 || g.splitk < 1 || (g.K / g.splitk) % 16 || g.K % g.splitk)
    return hipErrorInvalidValue;
  if (g.epi == EPI_SYMUPD && g.M != g.N) return hipErrorInvalidValue;
  const bool split = g.splitk > 1;
  GemmArgs run = g;
  if (split) {
    if (g.epi != EPI_COLSTORE || !partial_ws) return hipErrorInvalidValue;
    run.epi = EPI_PARTIAL;
    run.C = partial_ws;
  }
  int BM, BN;
  pick_tiles(run, BM, BN);
  const int64_t blocks = gemm_f64_blocks(run);
  hipError_t e = hipSuccess;
  if (run.epi == EPI_SYMUPD || run.epi == EPI_ADDROW || run.epi == EPI_RESID) {
    // n x n products: the order is a multiple of 256, always 128 x 128 tiles
    if (g.M % 128 || g.N % 128) return hipErrorInvalidValue;
    if (run.epi == EPI_SYMUPD && !run.a_kc && !run.b_kc)
      hipLaunchKernelGGL((k_gemm_f64<128, 128, false, false, EPI_SYMUPD>), dim3(blocks), dim3(256), 0, s, run);
    else if (run.epi == EPI_ADDROW && !run.a_kc && !run.b_kc)
      hipLaunchKernelGGL((k_gemm_f64<128, 128, false, false, EPI_ADDROW>), dim3(blocks), dim3(256), 0, s, run);
    else if (run.epi == EPI_RESID && run.a_kc && run.b_kc)
      hipLaunchKernelGGL((k_gemm_f64<128, 128, true, true, EPI_RESID>), dim3(blocks), dim3(256), 0, s, run);
    else if (run.epi == EPI_RESID && run.a_kc)  // I - A X for an X that is not symmetric
      hipLaunchKernelGGL((k_gemm_f64<128, 128, true, false, EPI_RESID>), dim3(blocks), dim3(256), 0, s, run);
    else
      return hipErrorInvalidValue;
  } else if (BM == 128 && BN == 128) e = launch_f64_epi<128, 128>(run, blocks, s);
  else if (BM == 64) e = launch_f64_epi<64, 64>(run, blocks, s);
  else if (BM == 128) e = launch_f64_epi<128, 32>(run, blocks, s);
  else if (BN == 128) e = launch_f64_epi<32, 128>(run, blocks, s);
  else e = launch_f64_epi<32, 32>(run, blocks, s);
  if (e != hipSuccess) return e;
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (g.mark && (e = hipEventRecord(g.mark, s)) != hipSuccess) return e;
  if (!split) return hipSuccess;
  return reduce_partials_f64(g, (const double*)partial_ws, s);
}

hipError_t reduce_partials_f64(const GemmArgs& g, const double* P, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partials_f64, dim3((unsigned)((g.M + 255) / 256), (unsigned)g.N), dim3(256), 0, s, g, P);
  return hipGetLastError();
}

// ------------------------------------------------------------- small kernels
__global__ void k_gather_cols_sym(const void* A, int a_dt, int64_t lda, const int32_t* C, int q, int64_t np,
                                  void* Y, int y_dt, int64_t ldy, double* G, int64_t ldg) {
  const int j = blockIdx.y;
  const int64_t row = (int64_t)C[j] * lda;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x)
    store_any(Y, y_dt, i + j * ldy, load_any(A, a_dt, row + i));
  if (G && blockIdx.x == 0)
    for (int b = threadIdx.x; b < q; b += blockDim.x) G[(int64_t)j * ldg + b] = load_any(A, a_dt, row + C[b]);
}

hipError_t gather_cols_sym(const void* A, int a_dt, int64_t lda, const int32_t* C, int q, int64_t np,
                           void* Y, int y_dt, int64_t ldy, double* G, int64_t ldg, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols_sym, dim3((unsigned)std::min<int64_t>(ceil_div(np, 256), 64), q), dim3(256), 0, s,
                     A, a_dt, lda, C, q, np, Y, y_dt, ldy, G, ldg);
  return hipGetLastError();
}

__global__ void k_gather_cols_gen(const void* L, int l_dt, int64_t ldl, const int32_t* C, int64_t np, void* S,
                                  int s_dt, int64_t lds) {
  const int j = blockIdx.y;
  const int64_t col = C[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x)
    store_any(S, s_dt, i + j * lds, load_any(L, l_dt, i * ldl + col));
}

hipError_t gather_cols_gen(const void* L, int l_dt, int64_t ldl, const int32_t* C, int q, int64_t np, void* S,
                           int s_dt, int64_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols_gen, dim3((unsigned)std::min<int64_t>(ceil_div(np, 256), 64), q), dim3(256), 0, s,
                     L, l_dt, ldl, C, np, S, s_dt, lds);
  return hipGetLastError();
}

// Per-block partial sums of (Sk - V)^2 over the n x q block.
// Per-workgroup sum of (S - V)^2 over rows blockIdx.x*256 + t (< n) and 16 columns
// from blockIdx.y*16 (< q); S dense (sk_dt) or coordinate (C: S[i][j] = [C_j == i]).
__global__ void k_est_partial(const void* Sk, int sk_dt, const int32_t* C, const void* V, int v_dt, int64_t ld,
                              int64_t n, int q, double* red) {
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j0 = blockIdx.y * 16;
  double s = 0;
  if (i < n) {
    for (int j = j0; j < j0 + 16 && j < q; ++j) {
      const double sv = C ? (C[j] == i ? 1.0 : 0.0) : load_any(Sk, sk_dt, i + j * ld);
      const double d = sv - load_any(V, v_dt, i + j * ld);
      s += d * d;
    }
  }
  const double t = block_sum_256(s, sh);
  if (threadIdx.x == 0) red[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// *out = scale * dscale * sum; with win, the value is also added to out[2] (the sum of
// the estimates since the host last cleared it).
__global__ void k_reduce_sum(const double* in, int64_t count, double* out, double scale, int* status,
                             const double* dscale, int win) {
  __shared__ double sh[4];
  double s = 0;
  for (int64_t e = threadIdx.x; e < count; e += 256) s += in[e];
  const double t = block_sum_256(s, sh);
  if (threadIdx.x == 0) {
    const double v = t * scale * (dscale ? *dscale : 1.0);
    *out = v;
    if (win) out[2] += v;
    if (status && !isfinite(t)) atomicCAS(status, 0, 4);
  }
}

hipError_t reduce_sum(const double* in, int64_t count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, in, count, out, 1.0, (int*)nullptr,
                     (const double*)nullptr, 0);
  return hipGetLastError();
}

hipError_t estimator(const void* Sk, int sk_dt, const int32_t* C, const void* V, int v_dt, int64_t ld, int64_t n,
                     int q, double scale, double* red, double* est, int* status, hipStream_t s, const double* dscale) {
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)((q + 15) / 16));
  hipLaunchKernelGGL(k_est_partial, grid, dim3(256), 0, s, Sk, sk_dt, C, V, v_dt, ld, n, q, red);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, red, (int64_t)grid.x * grid.y, est, scale, status,
                     dscale, 1);
  return hipGetLastError();
}

hipError_t reduce_sum_scaled(const double* in, int64_t count, double* out, double scale, int* status,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, in, count, out, scale, status, (const double*)nullptr, 1);
  return hipGetLastError();
}

__global__ void k_coord_wprime_fix(void* W, int w_dt, int64_t ld, const int32_t* C, int q, const double* GH,
                                   int64_t ldgh) {
  const int a = blockIdx.x;
  const int64_t row = C[a];
  for (int b = threadIdx.x; b < q; b += blockDim.x) {
    const int64_t idx = row + b * ld;
    const double v = load_any(W, w_dt, idx) - 0.5 * (a == b ? 1.0 : 0.0) - 0.5 * GH[(int64_t)a * ldgh + b];
    store_any(W, w_dt, idx, v);
  }
}

hipError_t coord_wprime_fix(void* W, int w_dt, int64_t ld, const int32_t* C, int q, const double* GH, int64_t ldgh,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_coord_wprime_fix, dim3(q), dim3(256), 0, s, W, w_dt, ld, C, q, GH, ldgh);
  return hipGetLastError();
}

__global__ void k_coord_add_rows(void* Qt, int dt, int64_t ld, const int32_t* C, int q, const double* M, int64_t ldm) {
  const int a = blockIdx.x;
  const int64_t row = C[a];
  for (int b = threadIdx.x; b < q; b += blockDim.x) {
    const int64_t idx = row + b * ld;
    store_any(Qt, dt, idx, load_any(Qt, dt, idx) + M[(int64_t)a * ldm + b]);
  }
}

hipError_t coord_add_rows(void* Qt, int dt, int64_t ld, const int32_t* C, int q, const double* M, int64_t ldm,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_coord_add_rows, dim3(q), dim3(256), 0, s, Qt, dt, ld, C, q, M, ldm);
  return hipGetLastError();
}

__global__ void k_pos_set(int32_t* pos, const int32_t* C, int q, int value_is_index) {
  for (int a = threadIdx.x; a < q; a += blockDim.x) pos[C[a]] = value_is_index ? a : -1;
}

// rows C_a: X[C_a, j] -= (R[a, j] + (j == C_b ? R[b, C_a] : 0)); the sum R[a,C_b] + R[b,C_a]
// is commutative, so the C x C block stays exactly symmetric.
__global__ void k_coord_rows(void* X, int x_dt, int64_t ldx, const int32_t* C, const int32_t* pos, int64_t np,
                             const void* R, int r_dt, int64_t ldr) {
  const int a = blockIdx.y;
  const int64_t ca = C[a];
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
    double d = load_any(R, r_dt, (int64_t)a * ldr + j);
    const int b = pos[j];
    if (b >= 0) d = d + load_any(R, r_dt, (int64_t)b * ldr + ca);
    const int64_t idx = ca * ldx + j;
    store_any(X, x_dt, idx, load_any(X, x_dt, idx) - d);
  }
}

// columns C_a at rows j not in C: X[j, C_a] = X[C_a, j]
__global__ void k_coord_mirror(void* X, int x_dt, int64_t ldx, const int32_t* C, const int32_t* pos, int64_t np) {
  const int a = blockIdx.y;
  const int64_t ca = C[a];
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
    if (pos[j] >= 0) continue;
    store_any(X, x_dt, j * ldx + ca, load_any(X, x_dt, ca * ldx + j));
  }
}

hipError_t coord_sym_update(void* X, int x_dt, int64_t ldx, const int32_t* C, int32_t* pos, int q, int64_t np,
                            const void* R, int r_dt, int64_t ldr, hipStream_t s) {
  hipLaunchKernelGGL(k_pos_set, dim3(1), dim3(256), 0, s, pos, C, q, 1);
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(np, 256), 64);
  hipLaunchKernelGGL(k_coord_rows, dim3(gx, q), dim3(256), 0, s, X, x_dt, ldx, C, (const int32_t*)pos, np, R, r_dt,
                     ldr);
  hipLaunchKernelGGL(k_coord_mirror, dim3(gx, q), dim3(256), 0, s, X, x_dt, ldx, C, (const int32_t*)pos, np);
  hipLaunchKernelGGL(k_pos_set, dim3(1), dim3(256), 0, s, pos, C, q, 0);
  return hipGetLastError();
}

__global__ void k_set_identity(void* X, int dt, int64_t ld, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    store_any(X, dt, i * ld + i, 1.0);
}

hipError_t set_identity(void* X, int dt, int64_t ld, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_set_identity, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 1024)), dim3(256), 0, s, X,
                     dt, ld, n);
  return hipGetLastError();
}

__global__ void k_copy_convert(const void* src, int s_dt, int64_t lds, void* dst, int d_dt, int64_t ldd, int64_t rows,
                               int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e % cols;
    store_any(dst, d_dt, i * ldd + j, load_any(src, s_dt, i * lds + j));
  }
}

hipError_t copy_convert(const void* src, int s_dt, int64_t lds, void* dst, int d_dt, int64_t ldd, int64_t rows,
                        int64_t cols, hipStream_t s) {
  const int64_t total = rows * cols;
  hipLaunchKernelGGL(k_copy_convert, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 8192)), dim3(256), 0, s,
                     src, s_dt, lds, dst, d_dt, ldd, rows, cols);
  return hipGetLastError();
}

__global__ void k_check_sym_finite(const void* A, int dt, int64_t lda, int64_t n, int sym, int* flag) {
  const int64_t total = n * n;
  int bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    const double v = load_any(A, dt, i * lda + j);
    if (!isfinite(v) || (sym && v != load_any(A, dt, j * lda + i))) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

hipError_t check_sym_finite(const void* A, int dt, int64_t lda, int64_t n, int* flag, hipStream_t s, bool sym) {
  const int64_t total = n * n;
  hipLaunchKernelGGL(k_check_sym_finite, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 8192)), dim3(256), 0,
                     s, A, dt, lda, n, sym ? 1 : 0, flag);
  return hipGetLastError();
}

// out = a X + b Y elementwise on column-major rows x cols panels with leading dimension ld.
__global__ void k_panel_axpby(const void* X, int xdt, double a, const void* Y, int ydt, double b, void* out, int odt,
                              int64_t rows, int64_t cols, int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = (e / rows) * ld + e % rows;
    store_any(out, odt, idx, a * load_any(X, xdt, idx) + b * load_any(Y, ydt, idx));
  }
}

hipError_t panel_axpby(const void* X, int xdt, double a, const void* Y, int ydt, double b, void* out, int odt,
                       int64_t rows, int64_t cols, int64_t ld, hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_axpby, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 8192)), dim3(256), 0, s, X,
                     xdt, a, Y, ydt, b, out, odt, rows, cols, ld);
  return hipGetLastError();
}

// dst[j*ldd + i] = src[i*lds + j] for i < rows, j < cols (with conversion).
__global__ void k_copy_transpose(const void* src, int s_dt, int64_t lds, void* dst, int d_dt, int64_t ldd,
                                 int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e % cols;
    store_any(dst, d_dt, j * ldd + i, load_any(src, s_dt, i * lds + j));
  }
}

hipError_t copy_transpose(const void* src, int s_dt, int64_t lds, void* dst, int d_dt, int64_t ldd, int64_t rows,
                          int64_t cols, hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_transpose, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 65536)), dim3(256), 0,
                     s, src, s_dt, lds, dst, d_dt, ldd, rows, cols);
  return hipGetLastError();
}

// ---------------------------------------------------------------- comparison methods
// Newton-Schulz and MR (Sec. 10) on n x n row-major FP64 matrices with leading dimension ld.

// w = A v, one wave per row.
__global__ __launch_bounds__(256) void k_gemv_f64(const double* A, int64_t ld, int64_t n, const double* v, double* w) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;  // uniform per wave; no barrier in this kernel
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s = fma(A[row * ld + j], v[j], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) w[row] = s;
}

// sigma = ||w||_2, v = w / sigma, *sigma_out = sigma (one workgroup, fixed summation order).
__global__ __launch_bounds__(1024) void k_normalize(const double* w, int64_t n, double* v, double* sigma_out) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s = fma(w[i], w[i], s);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double sig = sqrt(sh[0]);
  for (int64_t i = threadIdx.x; i < n; i += 1024) v[i] = w[i] / sig;
  if (threadIdx.x == 0) *sigma_out = sig;
}

__global__ void k_fill_f64(double* v, int64_t n, double x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) v[i] = x;
}

// X = 0.99 A^T / sigma^2 on the n x n block (Sec. 10, the Newton-Schulz start).
__global__ void k_ns_x0(const double* A, int64_t ld, int64_t n, const double* sigma, double* X) {
  const double s = *sigma;
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    X[i * ld + j] = (0.99 * A[j * ld + i]) / (s * s);
  }
}

// Per-block partial sums over the n x n block of row-major matrices:
//   mode 0: red[b] = sum (delta_ij - T_ij)^2                       (residual of T = A X)
//   mode 1: T := I - T in place, red[b] = sum of the new T_ij^2    (R = I - A X)
//   mode 2: red[2b] = sum T_ij Q_ij, red[2b+1] = sum Q_ij^2          (<R, Q>, <Q, Q>)
//   mode 3: red[2b] = trace T, red[2b+1] = sum T_ij^2                (Tr A, ||A||_F^2)
__global__ __launch_bounds__(256) void k_sums(double* T, const double* Q, int64_t ld, int64_t n, int mode, double* red) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n, idx = i * ld + j;
    const double t = T[idx];
    if (mode == 0) {
      const double d = (i == j ? 1.0 : 0.0) - t;
      a = fma(d, d, a);
    } else if (mode == 1) {
      const double r = (i == j ? 1.0 : 0.0) - t;
      T[idx] = r;
      a = fma(r, r, a);
    } else if (mode == 2) {
      const double qv = Q[idx];
      a = fma(t, qv, a);
      b = fma(qv, qv, b);
    } else {
      if (i == j) a += t;
      b = fma(t, t, b);
    }
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s0[threadIdx.x] += s0[threadIdx.x + st];
      s1[threadIdx.x] += s1[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (mode <= 1) {
      red[blockIdx.x] = s0[0];
    } else {
      red[2 * blockIdx.x] = s0[0];
      red[2 * blockIdx.x + 1] = s1[0];
    }
  }
}

// out[0], out[1] = sums of the pairs red[2b], red[2b+1] (one workgroup, fixed order).
__global__ __launch_bounds__(256) void k_reduce_pairs(const double* red, int nb, double* out) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += red[2 * i];
    b += red[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s0[threadIdx.x] += s0[threadIdx.x + st];
      s1[threadIdx.x] += s1[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

// X += (sc[0] / sc[1]) P on the whole ld x ld buffer (padding is zero in both).
__global__ void k_axpy_ratio(double* X, const double* P, int64_t total, const double* sc) {
  const double a = sc[0] / sc[1];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    X[e] = fma(a, P[e], X[e]);
}

// X = (sc[0] / sc[1]) I on the n x n block (Sec. 10, the MR start: Tr A / Tr(A A^T)).
__global__ void k_scaled_identity(double* X, int64_t ld, int64_t n, const double* sc) {
  const double c = sc[0] / sc[1];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    X[i * ld + i] = c;
}

int sums_blocks(int64_t n) { return (int)std::min<int64_t>(ceil_div(n * n, 256), 2048); }

hipError_t power_norm(const double* A, int64_t ld, int64_t n, int steps, double* v, double* w, double* sigma,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 1024)), dim3(256), 0, s, v, n,
                     1.0 / sqrt((double)n));
  for (int i = 0; i < steps; ++i) {
    hipLaunchKernelGGL(k_gemv_f64, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, A, ld, n, (const double*)v, w);
    hipLaunchKernelGGL(k_normalize, dim3(1), dim3(1024), 0, s, (const double*)w, n, v, sigma);
  }
  return hipGetLastError();
}

hipError_t ns_start(const double* A, int64_t ld, int64_t n, const double* sigma, double* X, hipStream_t s) {
  hipLaunchKernelGGL(k_ns_x0, dim3((unsigned)std::min<int64_t>(ceil_div(n * n, 256), 8192)), dim3(256), 0, s, A, ld, n,
                     sigma, X);
  return hipGetLastError();
}

hipError_t mat_sums(double* T, const double* Q, int64_t ld, int64_t n, int mode, double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_sums, dim3((unsigned)sums_blocks(n)), dim3(256), 0, s, T, Q, ld, n, mode, red);
  return hipGetLastError();
}

hipError_t reduce_pairs(const double* red, int nb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(256), 0, s, red, nb, out);
  return hipGetLastError();
}

hipError_t axpy_ratio(double* X, const double* P, int64_t total, const double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_ratio, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 8192)), dim3(256), 0, s, X, P,
                     total, sc);
  return hipGetLastError();
}

hipError_t fill_f64(double* v, int64_t count, double x, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)std::min<int64_t>(ceil_div(count, 256), 8192)), dim3(256), 0, s, v,
                     count, x);
  return hipGetLastError();
}

hipError_t scaled_identity(double* X, int64_t ld, int64_t n, const double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_scaled_identity, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 1024)), dim3(256), 0, s, X, ld,
                     n, sc);
  return hipGetLastError();
}

// ---------------------------------------------------------------- conjugate gradients
// y = M v for an n x n row-major M (FP32 or FP64, ld a multiple of 4), FP64 vectors; GEMV_RPW
// rows per wave, 16-byte loads of M.
template <class T>
__global__ __launch_bounds__(256) void k_gemv_rows(const T* M, int64_t ld, int64_t n, const double* v, double* y) {
  // GEMV_RPW consecutive rows per wave: each v[j..j+3] (8-byte aligned, loaded as scalars)
  // serves all of them, and the rows' sums are independent FMA chains
  constexpr int RPW = GEMV_RPW;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW;
  const int lane = threadIdx.x & 63;
  if (row0 >= n) return;  // uniform per wave; no barrier in this kernel
  const int nr = (int)min<int64_t>(RPW, n - row0);
  double s[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) s[r] = 0.0;
  const int64_t n4 = n / 4 * 4;
  for (int64_t j = 4 * lane; j < n4; j += 256) {
    const double v0 = v[j], v1 = v[j + 1], v2 = v[j + 2], v3 = v[j + 3];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      if (r < nr) {
        const T* Mr = M + (row0 + r) * ld;
        if constexpr (sizeof(T) == 4) {
          const float4 a = *(const float4*)(Mr + j);
          s[r] = fma((double)a.x, v0, s[r]);
          s[r] = fma((double)a.y, v1, s[r]);
          s[r] = fma((double)a.z, v2, s[r]);
          s[r] = fma((double)a.w, v3, s[r]);
        } else {
          const double2 a = *(const double2*)(Mr + j), b = *(const double2*)(Mr + j + 2);
          s[r] = fma(a.x, v0, s[r]);
          s[r] = fma(a.y, v1, s[r]);
          s[r] = fma(b.x, v2, s[r]);
          s[r] = fma(b.y, v3, s[r]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    if (r < nr) {
      const T* Mr = M + (row0 + r) * ld;
      for (int64_t j = n4 + lane; j < n; j += 64) s[r] = fma((double)Mr[j], v[j], s[r]);
    }
    double t = s[r];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0 && r < nr) y[row0 + r] = t;
  }
}

// Partial sums of y = M^T v: chunk c of the rows, columns j .. j + GEMV_T_COLS - 1 of thread
// t (j = GEMV_T_COLS t; vector loads, ld and j multiples of 4 / GEMV_T_COLS) -> part[c * n + j];
// each column's sum runs over the chunk's rows in order.
template <class T>
__global__ __launch_bounds__(256) void k_gemv_cols_part(const T* M, int64_t ld, int64_t n, const double* v, int64_t rows_per,
                                                        double* part) {
  constexpr int W = GEMV_T_COLS;
  const int64_t j = ((int64_t)blockIdx.x * 256 + threadIdx.x) * W;
  if (j >= n) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per, r1 = r0 + rows_per < n ? r0 + rows_per : n;
  double s[W];
#pragma unroll
  for (int c = 0; c < W; ++c) s[c] = 0.0;
  if (j + W <= n) {
#pragma unroll 4
    for (int64_t i = r0; i < r1; ++i) {
      const double vi = v[i];
      const T* Mi = M + i * ld + j;
      if constexpr (sizeof(T) == 4 && W == 4) {
        const float4 a = *(const float4*)Mi;
        s[0] = fma((double)a.x, vi, s[0]);
        s[1] = fma((double)a.y, vi, s[1]);
        s[2] = fma((double)a.z, vi, s[2]);
        s[3] = fma((double)a.w, vi, s[3]);
      } else if constexpr (sizeof(T) == 4 && W == 2) {
        const float2 a = *(const float2*)Mi;
        s[0] = fma((double)a.x, vi, s[0]);
        s[1] = fma((double)a.y, vi, s[1]);
      } else if constexpr (sizeof(T) == 8 && W % 2 == 0) {
#pragma unroll
        for (int c = 0; c < W; c += 2) {
          const double2 a = *(const double2*)(Mi + c);
          s[c] = fma(a.x, vi, s[c]);
          s[c + 1] = fma(a.y, vi, s[c + 1]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < W; ++c) s[c] = fma((double)Mi[c], vi, s[c]);
      }
    }
  } else {
    for (int64_t i = r0; i < r1; ++i)
      for (int c = 0; c < W && j + c < n; ++c) s[c] = fma((double)M[i * ld + j + c], v[i], s[c]);
  }
#pragma unroll
  for (int c = 0; c < W; ++c)
    if (j + c < n) part[(int64_t)blockIdx.y * n + j + c] = s[c];
}

__global__ void k_sum_chunks(const double* part, int64_t n, int chunks, double* y) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + j];
    y[j] = s;
  }
}

// out[0] = a . b (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void k_dot(const double* a, const double* b, int64_t n, double* out) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s = fma(a[i], b[i], s);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// alpha = sc[num] / sc[den]; x += alpha p; r -= alpha Ap.
__global__ void k_cg_xr(double* x, double* r, const double* p, const double* Ap, int64_t n, const double* sc, int num,
                        int den) {
  const double a = sc[num] / sc[den];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] = fma(a, p[i], x[i]);
    r[i] = fma(-a, Ap[i], r[i]);
  }
}

// beta = sc[num] / sc[den]; p = z + beta p.
__global__ void k_cg_p(double* p, const double* z, int64_t n, const double* sc, int num, int den) {
  const double bt = sc[num] / sc[den];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = fma(bt, p[i], z[i]);
}

hipError_t gemv(const void* M, int dt, int64_t ld, int64_t n, bool transpose, const double* v, double* y,
                double* part, hipStream_t s) {
  if (ld % 4) return hipErrorInvalidValue;
  if (!transpose) {
    if (dt == DT_F32)
      hipLaunchKernelGGL(k_gemv_rows<float>, dim3((unsigned)ceil_div(n, 4 * GEMV_RPW)), dim3(256), 0, s, (const float*)M,
                         ld, n, v, y);
    else
      hipLaunchKernelGGL(k_gemv_rows<double>, dim3((unsigned)ceil_div(n, 4 * GEMV_RPW)), dim3(256), 0, s,
                         (const double*)M, ld, n, v, y);
    return hipGetLastError();
  }
  const int chunks = GEMV_T_CHUNKS;
  const int64_t rows_per = ceil_div(n, chunks);
  const dim3 grid((unsigned)ceil_div(n, 256 * GEMV_T_COLS), (unsigned)chunks);
  if (dt == DT_F32)
    hipLaunchKernelGGL(k_gemv_cols_part<float>, grid, dim3(256), 0, s, (const float*)M, ld, n, v, rows_per, part);
  else
    hipLaunchKernelGGL(k_gemv_cols_part<double>, grid, dim3(256), 0, s, (const double*)M, ld, n, v, rows_per, part);
  hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 1024)), dim3(256), 0, s,
                     (const double*)part, n, chunks, y);
  return hipGetLastError();
}

hipError_t dot(const double* a, const double* b, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(1), dim3(1024), 0, s, a, b, n, out);
  return hipGetLastError();
}

hipError_t cg_xr(double* x, double* r, const double* p, const double* Ap, int64_t n, const double* sc, int num, int den,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_cg_xr, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 1024)), dim3(256), 0, s, x, r, p, Ap,
                     n, sc, num, den);
  return hipGetLastError();
}

hipError_t cg_p(double* p, const double* z, int64_t n, const double* sc, int num, int den, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 1024)), dim3(256), 0, s, p, z, n, sc,
                     num, den);
  return hipGetLastError();
}

// Dense coordinate sketch: S[i + j*ld] = (j < q && i == C[j]) for i < ld, j < qp.
__global__ void k_coord_dense(const int32_t* C, int q, void* S, int dt, int64_t ld, int64_t qp) {
  const int64_t total = ld * qp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / ld, i = e % ld;
    store_any(S, dt, e, (j < q && i == (int64_t)C[j]) ? 1.0 : 0.0);
  }
}

hipError_t coord_dense(const int32_t* C, int q, void* S, int dt, int64_t ld, int64_t qp, hipStream_t s) {
  const int64_t total = ld * qp;
  hipLaunchKernelGGL(k_coord_dense, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 8192)), dim3(256), 0, s, C,
                     q, S, dt, ld, qp);
  return hipGetLastError();
}


// ---------------------------------------------------------------- partition weights
// t_j = A_jj in FP64 for j < n (the weights of fixed RBFGS, and of AdaRBFGS at L = I).
__global__ void k_diag_weights(const void* A, int dt, int64_t ld, int64_t n, double* t) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) t[j] = load_any(A, dt, j * ld + j);
}

hipError_t diag_weights(const void* A, int dt, int64_t ld, int64_t n, double* t, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, dt, ld, n, t);
  return hipGetLastError();
}

// AdaRBFGS weight update t_j = (L^T A L)_jj from one step's panels (n x q column-major,
// leading dimension ld): with V = L^T Y and W = -L^T Y G^-1, sum_c V_jc W_jc = -||K_j||^2
// for K = L^T Y L_G^-T, and L+^T A L+ = L^T A L - K K^T + S~ (S~^T S~)^-1 S~^T, whose last
// term is the identity on the drawn block [C[0], C[0] + q) for a coordinate block.
template <class T>
__global__ __launch_bounds__(1024) void k_part_weights(const T* V, const T* W, int64_t ld, int64_t n, int q,
                                                       const int32_t* C, double* t) {
  // 64 rows per workgroup; wave g (of 16) sums columns g, g + 16, ... of its lane's row in two
  // chains, and the 16 partial sums are added in a fixed order (deterministic)
  __shared__ double part[16][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  double a0 = 0.0, a1 = 0.0;
  if (j < n) {
    int c = g;
    for (; c + 16 < q; c += 32) {
      a0 += (double)V[j + c * ld] * (double)W[j + c * ld];
      a1 += (double)V[j + (c + 16) * ld] * (double)W[j + (c + 16) * ld];
    }
    if (c < q) a0 += (double)V[j + c * ld] * (double)W[j + c * ld];
  }
  part[g][lane] = a0 + a1;
  __syncthreads();
  if (g == 0 && j < n) {
    double sum = 0.0;
    for (int w = 0; w < 16; ++w) sum += part[w][lane];
    const int64_t c0 = C[0];
    t[j] += sum + ((j >= c0 && j < c0 + q) ? 1.0 : 0.0);
  }
}

hipError_t part_weights(const void* V, const void* W, int dt, int64_t ld, int64_t n, int q, const int32_t* C, double* t,
                        hipStream_t s) {
  const dim3 grid((unsigned)((n + 63) / 64)), blk(1024);
  if (dt == DT_F32)
    hipLaunchKernelGGL(k_part_weights<float>, grid, blk, 0, s, (const float*)V, (const float*)W, ld, n, q, C, t);
  else if (dt == DT_F64)
    hipLaunchKernelGGL(k_part_weights<double>, grid, blk, 0, s, (const double*)V, (const double*)W, ld, n, q, C, t);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// t[C[c]] = sum_r P_rc Q_rc for the first q columns of two n x q column-major panels (one
// workgroup per column): the diagonal of L^T A L block by block, with P = L I_{:C}, Q = A P.
__global__ void k_col_dots(const void* P, const void* Q, int dt, int64_t ld, int64_t n, const int32_t* C, double* t) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) acc += load_any(P, dt, r + c * ld) * load_any(Q, dt, r + c * ld);
  const double v = block_sum_256(acc, sh);
  if (threadIdx.x == 0) t[C[c]] = v;
}

hipError_t col_dots(const void* P, const void* Q, int dt, int64_t ld, int64_t n, int q, const int32_t* C, double* t,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_col_dots, dim3((unsigned)q), dim3(256), 0, s, P, Q, dt, ld, n, C, t);
  return hipGetLastError();
}

// idx[c] = start + c, c < q.
__global__ void k_fill_block(int32_t* idx, int64_t start, int q) {
  for (int c = threadIdx.x; c < q; c += blockDim.x) idx[c] = (int32_t)(start + c);
}

hipError_t fill_block(int32_t* idx, int64_t start, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_block, dim3(1), dim3(256), 0, s, idx, start, q);
  return hipGetLastError();
}

}  // namespace rb
