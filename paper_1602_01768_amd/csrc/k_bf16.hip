// Mixed-precision GEMM on gfx950 bf16 MFMA (v_mfma_f32_32x32x16_bf16) with FP32
// accumulation.  Each FP32 operand is presented to the matrix cores as a sum of
// bf16 pieces (hi + lo, or hi + mid + lo), and the product is the sum of the piece
// products whose combined weight is at least 2^-(8*pmax): for two 2-piece operands
// hi*hi + hi*lo + lo*hi (3 passes); for a 3-piece operand times an exact bf16
// matrix all 3 passes are exact.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace rb {

namespace {

// Tall-skinny products: 32-deep k stages; two LDS buffers except for the product with an
// exact bf16 sketch (A S, L S~), where one buffer measured faster; wave grids of the
// 128 x 256 tile 2 x 4 (4 x 1 for the exact-sketch product, measured fastest).
constexpr int TS_BK = 32;
constexpr bool TS_LDB = true;
constexpr bool TS_LDB_AS = false;
#define RB_TS_WAVES256 2, 4
#define RB_TS_WAVES256_AS 4, 1
// LDS rows hold BK + 8 bf16 (16-byte aligned, rows 8 apart land on distinct banks)

template <int NP>
RB_DEV void split_n(float x, __bf16 (&o)[NP]) {
  if constexpr (NP == 1) {
    o[0] = f2bf(x);
  } else if constexpr (NP == 2) {
    split2(x, o[0], o[1]);
  } else {
    split3(x, o[0], o[1], o[2]);
  }
}

// Tall products whose split-K factor divides 8 take their tiles in the XCD-aware order of
// k_gemm_bf16; deeper splits (the q x q Grams) keep split index fastest.
RB_HD bool xcd_order(int splitk) { return splitk <= 8 && 8 % splitk == 0; }

// Loader for one operand tile of ROWS (m or n) x BK into LDS planes [NP][ROWS][PITCH].
template <int ROWS, int NP, int KIND, int NT, int BK>
struct TileLoader {
  static constexpr int PITCH = BK + 8;
  // registers held between the global load and the LDS store
  // F32_KC: float4 per thread; F32_MC: runs of 8 consecutive k of one row m (8 dword loads,
  // consecutive lanes on consecutive m, so each load instruction reads contiguous memory and
  // each 16-byte LDS store of a lane lands on rows one pitch apart: no bank conflicts);
  // BF16_MC: 4 x 4 micro-blocks
  static constexpr int MBLK = ROWS * BK / 16;
  static constexpr int MCU = (ROWS * (BK / 8) + NT - 1) / NT;  // F32_MC: 8-k runs per thread
  static constexpr int F4 = (KIND == OK_BF16_KC) ? 1
                            : (KIND == OK_F32_MC) ? 2 * MCU
                            : (KIND == OK_BF16_MC) ? 4 * ((MBLK + NT - 1) / NT)
                                                   : ROWS * BK / 4 / NT;
  static_assert(KIND != OK_BF16_MC || NP == 1, "an m-contiguous bf16 operand is exact: one piece");
  static constexpr int V8 = (KIND == OK_BF16_KC) ? (ROWS * (BK / 8) + NT - 1) / NT : 1;  // 16-byte chunks per plane
  float4 f[(F4 > 0 && KIND != OK_BF16_MC) ? F4 : 1];
  bf16x4 hm[KIND == OK_BF16_MC ? F4 : 1];
  bf16x8 h[NP][V8];

  RB_DEV void load(const void* base, int64_t ld, int64_t plane, int64_t r0, int64_t k0, int tid) {
    if constexpr (KIND == OK_F32_KC) {
      const float* A = (const float*)base;
#pragma unroll
      for (int i = 0; i < F4; ++i) {
        const int e = tid + NT * i;
        const int row = e / (BK / 4), c4 = (e % (BK / 4)) * 4;
        f[i] = *(const float4*)(A + (r0 + row) * ld + k0 + c4);
      }
    } else if constexpr (KIND == OK_F32_MC) {
      // run u: row m = u % ROWS, k = k0 + 8 (u / ROWS) .. + 7, one dword per k
      const float* A = (const float*)base;
#pragma unroll
      for (int i = 0; i < MCU; ++i) {
        const int u = tid + NT * i;
        if (ROWS * (BK / 8) % NT == 0 || u < ROWS * (BK / 8)) {
          const int m = u % ROWS, kg = u / ROWS;
          const float* src = A + (k0 + 8 * kg) * ld + r0 + m;
          f[2 * i] = make_float4(src[0], src[ld], src[2 * ld], src[3 * ld]);
          f[2 * i + 1] = make_float4(src[4 * ld], src[5 * ld], src[6 * ld], src[7 * ld]);
        }
      }
    } else if constexpr (KIND == OK_BF16_MC) {
      const __bf16* A = (const __bf16*)base;
#pragma unroll
      for (int i = 0; i < F4 / 4; ++i) {
        const int b = tid + NT * i;
        if (MBLK % NT == 0 || b < MBLK) {
          const int m4 = (b % (ROWS / 4)) * 4, kk = (b / (ROWS / 4)) * 4;
#pragma unroll
          for (int j = 0; j < 4; ++j) hm[4 * i + j] = *(const bf16x4*)(A + (k0 + kk + j) * ld + r0 + m4);
        }
      }
    } else {
      const __bf16* A = (const __bf16*)base;
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < V8; ++i) {
          const int e = tid + NT * i;
          if (ROWS * (BK / 8) % NT == 0 || e < ROWS * (BK / 8)) {
            const int row = e / (BK / 8), c8 = (e % (BK / 8)) * 8;
            h[p][i] = *(const bf16x8*)(A + p * plane + (r0 + row) * ld + k0 + c8);
          }
        }
    }
  }

  RB_DEV void store(__bf16* lds, int tid) {
    if constexpr (KIND == OK_F32_KC) {
#pragma unroll
      for (int i = 0; i < F4; ++i) {
        const int e = tid + NT * i;
        const int row = e / (BK / 4), c4 = (e % (BK / 4)) * 4;
        __bf16 p0[NP], p1[NP], p2[NP], p3[NP];
        split_n<NP>(f[i].x, p0);
        split_n<NP>(f[i].y, p1);
        split_n<NP>(f[i].z, p2);
        split_n<NP>(f[i].w, p3);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          bf16x4 v = {p0[p], p1[p], p2[p], p3[p]};
          *(bf16x4*)(lds + (p * ROWS + row) * PITCH + c4) = v;
        }
      }
    } else if constexpr (KIND == OK_F32_MC) {
      // run u: one 16-byte store per piece into row m, k columns 8 kg .. 8 kg + 7
#pragma unroll
      for (int i = 0; i < MCU; ++i) {
        const int u = tid + NT * i;
        if (ROWS * (BK / 8) % NT == 0 || u < ROWS * (BK / 8)) {
          const int m = u % ROWS, kg = u / ROWS;
          const float v[8] = {f[2 * i].x, f[2 * i].y, f[2 * i].z, f[2 * i].w,
                              f[2 * i + 1].x, f[2 * i + 1].y, f[2 * i + 1].z, f[2 * i + 1].w};
          __bf16 pc[8][NP];
#pragma unroll
          for (int e = 0; e < 8; ++e) split_n<NP>(v[e], pc[e]);
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            bf16x8 w;
#pragma unroll
            for (int e = 0; e < 8; ++e) w[e] = pc[e][p];
            *(bf16x8*)(lds + (p * ROWS + m) * PITCH + 8 * kg) = w;
          }
        }
      }
    } else if constexpr (KIND == OK_BF16_MC) {
      // transpose the 4 x 4 bf16 micro-block: LDS row m gets k = kk..kk+3
#pragma unroll
      for (int i = 0; i < F4 / 4; ++i) {
        const int b = tid + NT * i;
        if (MBLK % NT == 0 || b < MBLK) {
          const int m4 = (b % (ROWS / 4)) * 4, kk = (b / (ROWS / 4)) * 4;
          const bf16x4* hb = &hm[4 * i];
#pragma unroll
          for (int mm = 0; mm < 4; ++mm) {
            bf16x4 v = {hb[0][mm], hb[1][mm], hb[2][mm], hb[3][mm]};
            *(bf16x4*)(lds + (m4 + mm) * PITCH + kk) = v;
          }
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < V8; ++i) {
          const int e = tid + NT * i;
          if (ROWS * (BK / 8) % NT == 0 || e < ROWS * (BK / 8)) {
            const int row = e / (BK / 8), c8 = (e % (BK / 8)) * 8;
            *(bf16x8*)(lds + (p * ROWS + row) * PITCH + c8) = h[p][i];
          }
        }
    }
  }
};

// Tall-skinny product, split-K: FP32 partial sums of K chunk kc of output tile (mt, nt).
// NT = 64 * WAVES_M * WAVES_N threads; wave tile WM x WN of 32 x 32 blocks.
// v_mfma_f32_32x32x16_bf16: lane l holds A(l%32, 8*(l/32) .. +7), B(8*(l/32) .. +7, l%32);
// output column l%32, rows 8*(r/4) + 4*(l/32) + r%4 for r = 0..15.
// LDB: two LDS buffers (one barrier per k tile, the next tile staged during the MFMAs);
// otherwise one buffer with the next tile's global loads in flight during the MFMAs.
// Launch bounds ask for two waves per SIMD (<= 256 VGPRs).
template <int BM, int BN, int WAVES_M, int WAVES_N, int NA, int NB, int PMAX, int AK, int BKD, bool LDB, int BK>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N, 2) void k_gemm_bf16(GemmArgs g) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int PITCH = BK + 8;
  constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int LOOP_E = (NA * BM + NB * BN) * PITCH;  // bf16 elements of one buffer
  __shared__ __attribute__((aligned(16))) __bf16 smem[(LDB ? 2 : 1) * LOOP_E];
  __bf16* As = smem;
  __bf16* Bs = smem + NA * BM * PITCH;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const int64_t MT = g.M / BM;
  int kc;
  int64_t mt, nt;
  if (!xcd_order(g.splitk)) {
    const int64_t bid = blockIdx.x;
    kc = (int)(bid % g.splitk);
    mt = (bid / g.splitk) % MT;
    nt = (bid / g.splitk) / MT;
  } else {
    // blockIdx % 8 is the XCD: it fixes the K chunk (XCDs of one chunk share its slice of the
    // panel in their L2s) and a residue class of row tiles; within an XCD the column tiles of
    // one row tile are consecutive, so the row tile of the n x n operand is read from HBM once
    // and the next column tile finds it in the same L2
    const int x = (int)(blockIdx.x % 8), G = 8 / g.splitk;
    const int64_t l = blockIdx.x / 8, NTT = g.N / BN;
    kc = x % g.splitk;
    nt = l % NTT;
    mt = (l / NTT) * G + x / g.splitk;
    if (mt >= MT) return;
  }
  const int64_t kchunk = g.K / g.splitk;
  const int64_t kbeg = kc * kchunk, kend = kbeg + kchunk;
  const int64_t m0 = mt * BM, n0 = nt * BN;

  f32x16 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  // MFMAs of one 16-wide k sub-step s of the tile held in LDS at (As_, Bs_); piece
  // products ordered smallest first.
  auto substep = [&](const __bf16* As_, const __bf16* Bs_, int s) {
    bf16x8 av[NA][FM], bv[NB][FN];
    const int kofs = s * 16 + 8 * (lane >> 5);
#pragma unroll
    for (int p = 0; p < NA; ++p)
#pragma unroll
      for (int a = 0; a < FM; ++a)
        av[p][a] = *(const bf16x8*)(As_ + (p * BM + wm * WM + a * 32 + (lane & 31)) * PITCH + kofs);
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
      for (int b = 0; b < FN; ++b)
        bv[p][b] = *(const bf16x8*)(Bs_ + (p * BN + wn * WN + b * 32 + (lane & 31)) * PITCH + kofs);
#pragma unroll
    for (int lvl = PMAX; lvl >= 0; --lvl)
#pragma unroll
      for (int pa = 0; pa < NA; ++pa) {
        const int pb = lvl - pa;
        if (pb < 0 || pb >= NB) continue;
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[pa][a], bv[pb][b], acc[a][b], 0, 0, 0);
      }
  };

  TileLoader<BM, NA, AK, NT, BK> la;
  TileLoader<BN, NB, BKD, NT, BK> lb;
  la.load(g.A, g.lda, g.a_plane, m0, kbeg, tid);
  lb.load(g.B, g.ldb, g.b_plane, n0, kbeg, tid);
  if constexpr (LDB) {
    // While the MFMAs of tile t run on buffer t&1, tile t+1 (already in registers) is
    // split into the other buffer and the global loads of tile t+2 start.  Buffer
    // (t+1)&1 was last read in iteration t-1, which the barrier closing it has finished.
    la.store(As, tid);
    lb.store(Bs, tid);
    if (kbeg + BK < kend) {
      la.load(g.A, g.lda, g.a_plane, m0, kbeg + BK, tid);
      lb.load(g.B, g.ldb, g.b_plane, n0, kbeg + BK, tid);
    }
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
      const __bf16* Ac = As + cur * LOOP_E;
      const __bf16* Bc = Bs + cur * LOOP_E;
      substep(Ac, Bc, 0);
      if (k0 + BK < kend) {
        la.store(As + (cur ^ 1) * LOOP_E, tid);
        lb.store(Bs + (cur ^ 1) * LOOP_E, tid);
        if (k0 + 2 * BK < kend) {
          la.load(g.A, g.lda, g.a_plane, m0, k0 + 2 * BK, tid);
          lb.load(g.B, g.ldb, g.b_plane, n0, k0 + 2 * BK, tid);
        }
      }
#pragma unroll
      for (int s = 1; s < BK / 16; ++s) substep(Ac, Bc, s);
      __syncthreads();
      cur ^= 1;
    }
  } else {
    // one buffer: stage the registers of tile k0 into LDS, start the global loads of
    // tile k0 + BK into the same registers, then run the MFMAs on LDS
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
      __syncthreads();
      la.store(As, tid);
      lb.store(Bs, tid);
      __syncthreads();
      if (k0 + BK < kend) {
        la.load(g.A, g.lda, g.a_plane, m0, k0 + BK, tid);
        lb.load(g.B, g.ldb, g.b_plane, n0, k0 + BK, tid);
      }
#pragma unroll
      for (int s = 0; s < BK / 16; ++s) substep(As, Bs, s);
    }
  }

  // column-major partial sums of split kc: P[kc][n * M + m]; a lane holds rows
  // 8 g + lr + j (j = 0..3) of column lc, one 16-byte store per g.  The lane offsets
  // are recomputed here from an opaque copy of the lane index, so that the compiler
  // does not hold these addresses through the k loop.
  int ln = lane;
  asm volatile("" : "+v"(ln));
  const uint32_t plr = (ln >> 5) * 4, plc = ln & 31;
  float* P = (float*)g.C + (int64_t)kc * g.M * g.N + (n0 + wn * WN) * g.M + (m0 + wm * WM);
  const uint32_t ldp = (uint32_t)g.M;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
        *(float4*)(P + (b * 32 + plc) * ldp + a * 32 + q4 * 8 + plr) =
            make_float4(acc[a][b][4 * q4], acc[a][b][4 * q4 + 1], acc[a][b][4 * q4 + 2], acc[a][b][4 * q4 + 3]);
}

// C[m + n*ldc] = c2 * sum_k P[k][n*M + m] (+ c0 * B0[m + n*ld01]); grid (M / 1024, N),
// four consecutive m per thread.  With est_red: per-workgroup sum of (est_S - C)^2.
__global__ __launch_bounds__(256) void k_reduce_partials_f32(GemmArgs g, const float* P) {
  const int64_t n = blockIdx.y, m = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  double e2 = 0.0;
  if (m < g.M) {
    const int64_t MN = g.M * g.N, o = n * g.M + m;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int k = 0; k < g.splitk; ++k) {
      const float4 v = *(const float4*)(P + (int64_t)k * MN + o);
      s0 += v.x; s1 += v.y; s2 += v.z; s3 += v.w;
    }
    s0 *= g.c2; s1 *= g.c2; s2 *= g.c2; s3 *= g.c2;
    if (g.B0) {
      const float* b = (const float*)g.B0 + m + n * g.ld01;
      s0 += g.c0 * (double)b[0]; s1 += g.c0 * (double)b[1]; s2 += g.c0 * (double)b[2]; s3 += g.c0 * (double)b[3];
    }
    if (g.B1) {
      double b0, b1, b2, b3;
      if (g.b1_dt == DT_BF16) {
        const __bf16* b = (const __bf16*)g.B1 + m + n * g.ld01;
        b0 = (float)b[0]; b1 = (float)b[1]; b2 = (float)b[2]; b3 = (float)b[3];
      } else {
        const float* b = (const float*)g.B1 + m + n * g.ld01;
        b0 = b[0]; b1 = b[1]; b2 = b[2]; b3 = b[3];
      }
      s0 += g.c1 * b0; s1 += g.c1 * b1; s2 += g.c1 * b2; s3 += g.c1 * b3;
    }
    if (g.c_dt == DT_F64) {
      double* c = (double*)g.C + m + n * g.ldc;
      c[0] = s0; c[1] = s1; c[2] = s2; c[3] = s3;
      return;  // (no estimator on this path)
    }
    const float4 r = {(float)s0, (float)s1, (float)s2, (float)s3};
    *(float4*)((float*)g.C + m + n * g.ldc) = r;
    if (g.est_red) {
      const __bf16* sv = g.est_S + m + n * g.ldc;
      const double d0 = (double)(float)sv[0] - r.x, d1 = (double)(float)sv[1] - r.y;
      const double d2 = (double)(float)sv[2] - r.z, d3 = (double)(float)sv[3] - r.w;
      e2 = (d0 * d0 + d1 * d1) + (d2 * d2 + d3 * d3);
    }
  }
  if (g.est_red) {
    __shared__ double sh[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) g.est_red[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  }
}

// Column-major FP32 panel -> row-major bf16 hi/lo planes, through a 32 x 64 LDS tile.
// 64 rows x 32 columns per block: wave w takes columns c0 + 8 w .. + 7 (one 16-byte store per
// plane and row), lane l row r0 + l (the loads of one column coalesced across the wave); with
// mid, three pieces (hi, mid, lo)
__global__ __launch_bounds__(256) void k_pack_split2(const float* __restrict__ in, int64_t ld_in, int64_t rows,
                                                     int64_t cols, __bf16* __restrict__ hi, __bf16* __restrict__ lo,
                                                     int64_t ld_out, int64_t col_off, int tile_log2,
                                                     __bf16* __restrict__ mid) {
  const int64_t r = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t c0 = (int64_t)blockIdx.y * 32 + 8 * (threadIdx.x >> 6);
  if (r >= rows || c0 >= cols) return;
  const int m = cols - c0 < 8 ? (int)(cols - c0) : 8;
  bf16x8 h, md, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float v = e < m ? in[r + (c0 + e) * ld_in] : 0.0f;
    __bf16 he, me, le;
    if (mid) {
      split3(v, he, me, le);
    } else {
      split2(v, he, le);
      me = he;
    }
    h[e] = he;
    md[e] = me;
    l[e] = le;
  }
  const int64_t c = col_off + c0;
  int64_t o;
  if (tile_log2 >= 0) {
    const int64_t tile = (int64_t)1 << tile_log2;
    o = (r >> tile_log2) * tile * ld_out + (c >> 5) * tile * 32 + (r & (tile - 1)) * 32 + (c & 31);
  } else {
    o = r * ld_out + c;
  }
  if (m == 8 && o % 8 == 0) {
    *(bf16x8*)(hi + o) = h;
    *(bf16x8*)(lo + o) = l;
    if (mid) *(bf16x8*)(mid + o) = md;
  } else {
    for (int e = 0; e < m; ++e) {
      hi[o + e] = h[e];
      lo[o + e] = l[e];
      if (mid) mid[o + e] = md[e];
    }
  }
}

template <int BN, int WAVES_M, int WAVES_N, int NA, int NB, int PMAX, int AK, int BKD, bool LDB>
void launch_ts(const GemmArgs& g, int64_t blocks, hipStream_t s) {
  // two LDS buffers when asked for and they fit in the 160 KiB of LDS
  constexpr bool ldb = LDB && 2 * (NA * 128 + NB * BN) * (TS_BK + 8) * 2 <= 160 * 1024;
  hipLaunchKernelGGL((k_gemm_bf16<128, BN, WAVES_M, WAVES_N, NA, NB, PMAX, AK, BKD, ldb, TS_BK>),
                     dim3(blocks), dim3(64 * WAVES_M * WAVES_N), 0, s, g);
}

template <int NA, int NB, int PMAX, int AK, int BKD, bool LDB, int WM256, int WN256>
hipError_t launch_tall(const GemmArgs& g, int bn, int64_t blocks, hipStream_t s) {
  switch (bn) {
    case 256: launch_ts<256, WM256, WN256, NA, NB, PMAX, AK, BKD, LDB>(g, blocks, s); break;
    case 128: launch_ts<128, 2, 2, NA, NB, PMAX, AK, BKD, LDB>(g, blocks, s); break;
    case 64: launch_ts<64, 2, 2, NA, NB, PMAX, AK, BKD, LDB>(g, blocks, s); break;
    default: launch_ts<32, 4, 1, NA, NB, PMAX, AK, BKD, LDB>(g, blocks, s); break;
  }
  return hipGetLastError();
}

int pick_bn_auto(int64_t N);
int pick_bn(const GemmArgs& g) {
  if (g.bn == 256 || g.bn == 128 || g.bn == 64 || g.bn == 32) return (g.N % g.bn == 0) ? g.bn : pick_bn_auto(g.N);
  return pick_bn_auto(g.N);
}
int pick_bn_auto(int64_t N) {
  if (N % 256 == 0) return 256;
  if (N % 128 == 0) return 128;
  if (N % 64 == 0) return 64;
  return 32;
}

}  // namespace

// The symmetric update with wide panels (K = 2q >= 256, where the panel loads dominate) takes
// 256 x 256 tiles where there are still at least 1024 of them (four per CU): half the panel
// bytes per entry of X (n = 32768, q = 512: 4.94 -> 4.63 ms with row-major panels; at n = 16384,
// q = 256 the fixed step is the same with either size since the panels are tile-major); the
// full-square update of AdaRBFGS stays on 128 x 128 tiles (256: 0.57 -> 0.64 ms at n = 16384).
int bf16_square_tile(int64_t M, int64_t K, int epi) {
  if (M % 256 || K < 256 || epi != EPI_SYMUPD) return 128;
  const int64_t T = M / 256;
  return T * (T + 1) / 2 >= 1024 ? 256 : 128;
}

int64_t gemm_bf16_blocks(const MixedGemm& mg) {
  const GemmArgs& g = mg.g;
  if (g.epi == EPI_SYMUPD || g.epi == EPI_ADDROW) {
    const int64_t T = g.M / (g.bn == 256 ? 256 : 128);
    const int64_t NTT = g.tiles ? g.ntiles : (g.epi == EPI_SYMUPD ? T * (T + 1) / 2 : T * T);
    return (NTT + 7) / 8 * 8;
  }
  const int64_t MT = g.M / 128, NTT = g.N / pick_bn(g);
  if (!xcd_order(g.splitk)) return MT * NTT * g.splitk;
  const int64_t G = 8 / g.splitk;
  return 8 * ((MT + G - 1) / G) * NTT;  // row tiles beyond MT return at once
}

hipError_t gemm_bf16(const MixedGemm& mg, void* partial_ws, hipStream_t s) {
  const GemmArgs& g = mg.g;
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
  if (g.M % 128 || g.N % 32 || g.splitk < 1) return hipErrorInvalidValue;
  if (g.epi == EPI_SYMUPD || g.epi == EPI_ADDROW) {
    // square updates: operands pre-split into 2 bf16 planes, loaded straight into LDS
    const bool two = mg.na == 2 && mg.nb == 2 && mg.pmax == 1 && g.upd_pieces == 2;
    const bool three = mg.na == 3 && mg.nb == 3 && mg.pmax == 2 && g.upd_pieces == 3;
    if (g.N % 128 || g.K % 32 || mg.a_kind != OK_BF16_KC || mg.b_kind != OK_BF16_KC || !(two || three) ||
        g.splitk != 1)
      return hipErrorInvalidValue;
    return symupd_bf16_dma(g, gemm_bf16_blocks(mg), s);
  }
  if (g.K % (TS_BK * g.splitk)) return hipErrorInvalidValue;
  if (g.epi != EPI_COLSTORE || !partial_ws) return hipErrorInvalidValue;
  GemmArgs run = g;
  run.epi = EPI_PARTIAL;
  run.C = partial_ws;
  hipError_t e;
  if (tall_stream_supported(mg)) {
    if ((e = tall_stream(run, mg, s)) != hipSuccess) return e;
    if (g.mark && (e = hipEventRecord(g.mark, s)) != hipSuccess) return e;
    return reduce_partials_f32(g, (const float*)partial_ws, s);
  }
  const int bn = pick_bn(g);
  const int64_t blocks = gemm_bf16_blocks(mg);
#define RB_TALL(NA_, NB_, PM_, AK_, BK_, LDB_, WAVES256_)                                              \
  if (mg.na == NA_ && mg.nb == NB_ && mg.pmax == PM_ && mg.a_kind == AK_ && mg.b_kind == BK_)         \
    e = launch_tall<NA_, NB_, PM_, AK_, BK_, LDB_, WAVES256_>(run, bn, blocks, s);                    \
  else
  RB_TALL(3, 1, 2, OK_F32_KC, OK_BF16_KC, TS_LDB_AS, RB_TS_WAVES256_AS)  // A S, exact bf16 sketch; L S~
  RB_TALL(2, 2, 1, OK_F32_KC, OK_F32_KC, TS_LDB, RB_TS_WAVES256)        // X Y
  RB_TALL(3, 2, 2, OK_F32_KC, OK_F32_KC, TS_LDB, RB_TS_WAVES256)        // A S with S = L S~ (FP32)
  RB_TALL(2, 3, 2, OK_F32_MC, OK_F32_KC, TS_LDB, RB_TS_WAVES256)        // L^T Y
  RB_TALL(2, 2, 1, OK_F32_MC, OK_F32_KC, TS_LDB, RB_TS_WAVES256)        // X^T P (row variants)
  RB_TALL(3, 1, 2, OK_F32_MC, OK_BF16_KC, TS_LDB_AS, RB_TS_WAVES256_AS)  // A^T S (Kaczmarz)
  // q-sized products: one LDS buffer, so that they share CUs with the n x n products
  RB_TALL(1, 3, 2, OK_BF16_KC, OK_F32_KC, false, RB_TS_WAVES256)  // G = S^T Y
  RB_TALL(1, 3, 2, OK_BF16_MC, OK_F32_KC, false, RB_TS_WAVES256)  // U = S G^-1
  RB_TALL(3, 3, 2, OK_F32_KC, OK_F32_KC, false, RB_TS_WAVES256)   // H = Y^T V
  RB_TALL(3, 3, 2, OK_F32_MC, OK_F32_KC, false, RB_TS_WAVES256)   // U H
  return hipErrorInvalidValue;
#undef RB_TALL
  if (e != hipSuccess) return e;
  if (g.mark && (e = hipEventRecord(g.mark, s)) != hipSuccess) return e;
  return reduce_partials_f32(g, (const float*)partial_ws, s);
}

int64_t reduce_blocks_f32(const GemmArgs& g) { return (g.M + 1023) / 1024 * g.N; }

hipError_t reduce_partials_f32(const GemmArgs& g, const float* P, hipStream_t s) {
  if (g.M % 4 || g.ldc % 4 || ((g.B0 || g.B1) && g.ld01 % 4) || (g.c_dt == DT_F64 && g.est_red))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_partials_f32, dim3((unsigned)((g.M + 1023) / 1024), (unsigned)g.N), dim3(256), 0, s, g,
                     P);
  return hipGetLastError();
}

int64_t make_tile_order(int T, int S, bool lower, int2* out) {
  int64_t c = 0;
  for (int I = 0; I < T; I += S)
    for (int J = 0; J <= (lower ? I : T - 1); J += S)
      for (int i = I; i < I + S && i < T; ++i)
        for (int j = J; j < J + S && j < T; ++j)
          if (!lower || j <= i) {
            if (out) out[c] = make_int2(i, j);
            ++c;
          }
  return c;
}

hipError_t pack_split2(const float* in, int64_t ld_in, int64_t rows, int64_t cols, __bf16* hi, __bf16* lo,
                       int64_t ld_out, int64_t col_off, hipStream_t s, int64_t tile, __bf16* mid) {
  // tile-major: a power-of-two tile, whole tiles, 32-column stages (a thread's 8 columns then
  // stay in one stage)
  if (tile && (tile & (tile - 1) || rows % tile || ld_out % 32 || col_off % 32)) return hipErrorInvalidValue;
  const int tile_log2 = tile ? __builtin_ctzll((unsigned long long)tile) : -1;
  dim3 grid((unsigned)ceil_div(rows, 64), (unsigned)ceil_div(cols, 32));
  hipLaunchKernelGGL(k_pack_split2, grid, dim3(256), 0, s, in, ld_in, rows, cols, hi, lo, ld_out, col_off, tile_log2,
                     mid);
  return hipGetLastError();
}

}  // namespace rb
