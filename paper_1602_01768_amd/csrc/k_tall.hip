// Tall-skinny split-bf16 products P = A B with A an n x n FP32 matrix (A, X or L, k-contiguous
// rows) and B an n x q panel already split into bf16 planes (B^T rows, k-contiguous): the
// n x n-by-n x q products of eq. (qunac) and eq. (Cholimprov) for q a multiple of 128.
//
// A is the one operand streamed from HBM, and no two waves need the same rows of it: each of
// the 8 waves of a workgroup owns 32 rows of a 256-row tile and loads them straight into
// registers in the MFMA operand layout (no LDS), three k tiles ahead, and splits them into
// bf16 pieces right before its MFMAs -- every element of A is loaded and split exactly once.
// A is read as stored (four 16-byte loads per lane and tile) or transposed, A = M^T (L^T Y of
// AdaRBFGS, X^T P of the row variants): then each lane takes its 16 values of column m with
// one 4-byte load per k, the 32 lanes of a half-wave reading 128 contiguous bytes of a row.
// A symmetric A held on its lower 128 x 128 tiles only (X of the fixed method; diagonal tiles
// whole and exactly symmetric) is read as stored left of the workgroup's switch column and
// transposed from the lower tiles right of it, each k loop running without a choice per tile.
// The B tile (all q columns, or 256 of them) is shared by the 8 waves and travels from memory
// straight into LDS (global_load_lds_dwordx4) through a ring of three stages, one barrier per
// 32-deep k tile; B's planes are tile-major (split_planes), so a stage is one contiguous
// block and every load reads 1 KB of whole 128-byte lines.  The k order inside a tile is permuted to match the registers a lane holds
// (lane l loads k = 16 (l / 32) .. + 15 of its row; sub-step s feeds the MFMA with
// k = 16 (l / 32) + 8 s .. + 7), and B is read from LDS with the same permutation.
//
// Split-K partial sums of chunk kc go to P[kc][n * M + m] (column-major), summed afterwards by
// reduce_partials_f32.
#include "common.hpp"
#include "kernels.hpp"

namespace rb {

namespace {

typedef __attribute__((address_space(3))) void lds_void;

constexpr int TL_BM = 256;  // rows per workgroup (8 waves x 32)
constexpr int TL_BK = 32;   // k per tile

// s_waitcnt immediate for "at most n vector-memory operations outstanding" (vmcnt in bits
// 3:0 and 15:14, expcnt and lgkmcnt at their maxima) and for "no LDS operation outstanding"
constexpr int tl_vmcnt(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
constexpr int tl_lgkm0() { return 15 | (3 << 14) | (7 << 4); }

template <int NP>
RB_DEV void split_vec(const float (&x)[8], bf16x8 (&o)[NP]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    if constexpr (NP == 1) {
      o[0][e] = f2bf(x[e]);
    } else if constexpr (NP == 2) {
      __bf16 h, l;
      split2(x[e], h, l);
      o[0][e] = h;
      o[1][e] = l;
    } else {
      __bf16 h, m, l;
      split3(x[e], h, m, l);
      o[0][e] = h;
      o[1][e] = m;
      o[2][e] = l;
    }
  }
}

// AM: 0 as stored, 1 transposed, 2 symmetric on its lower 128 x 128 tiles
template <int BN, int NA, int NB, int PMAX, int AM>
__global__ __launch_bounds__(512, 1) void k_tall_stream(GemmArgs g) {
  constexpr int NW = 8, FN = BN / 32;
  constexpr int ROWB = TL_BK * 2;          // bytes of one B row of one piece in a stage (64)
  constexpr int CHUNKS = ROWB / 16;        // 16-byte chunks per row (4)
  constexpr int RPB = 128 / ROWB;          // rows per 128-byte bank period (2)
  constexpr int PLB = BN * ROWB;           // bytes of one piece
  constexpr int STB = NB * PLB;            // bytes of one stage
  constexpr int D = STB / (NW * 1024);     // 1 KB DMA loads per wave per stage
  static_assert(STB % (NW * 1024) == 0 && PLB % 1024 == 0, "whole 1 KB loads per wave");
  __shared__ __attribute__((aligned(1024))) char st0[STB];
  __shared__ __attribute__((aligned(1024))) char st1[STB];
  __shared__ __attribute__((aligned(1024))) char st2[STB];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  // tile: blockIdx % 8 is the XCD; it fixes the K chunk (the XCDs of one chunk share its
  // slice of B in their L2s) and a residue class of row tiles, and the column tiles of one
  // row tile run consecutively on one XCD (the row tile of A is read from HBM once).  The
  // K chunks are interleaved in runs of R = 8 (or 4, 2, 1: the largest dividing the chunk's
  // tile count) 32-deep k tiles: chunk kc takes runs kc, kc + splitk, ..., so that the
  // workgroups of one row tile, which run at the same time on different XCDs, read
  // neighbouring pieces of the same rows of A and HBM serves longer runs per row than from
  // contiguous chunks (A read alone in 256 x 32 tiles: 3.8 TB/s from contiguous chunks, 4.3
  // from eight chunks interleaved tile by tile; in the products, runs of 8 tiles beat runs
  // of 1, 2 and 4, whose B rows share 128-byte lines between XCDs).
  const int64_t MT = (g.M + TL_BM - 1) / TL_BM, NTT = g.N / BN;
  const int x = (int)(blockIdx.x % 8), G = 8 / g.splitk;
  const int64_t l = blockIdx.x / 8;
  const int kc = x % g.splitk;
  const int64_t nt = l % NTT, mt = (l / NTT) * G + x / g.splitk;
  if (mt >= MT) return;
  const int nk = (int)(g.K / ((int64_t)TL_BK * g.splitk));
  // k of tile t: kbeg + (t / R) kper + (t % R) TL_BK, R = 2^lr
  const int lr = nk % 8 == 0 ? 3 : nk % 4 == 0 ? 2 : nk % 2 == 0 ? 1 : 0;
  const int64_t kbeg = ((int64_t)kc * TL_BK) << lr, kper = ((int64_t)TL_BK * g.splitk) << lr;
  auto koff = [&](int t) -> int64_t { return (int64_t)(t >> lr) * kper + (int64_t)(t & ((1 << lr) - 1)) * TL_BK; };
  const int64_t m0 = mt * TL_BM, n0 = nt * BN;
  const int64_t mw = m0 + 32 * wave;  // this wave's rows
  const bool rows_ok = mw < g.M;      // (M is a multiple of 32)

  // The body for the ways of reading A, chosen once per workgroup: with X on its lower tiles
  // the tiles of a chunk left of the workgroup's switch column are read as stored and the
  // rest transposed, in two k loops of one way each.  A choice made per tile inside the loop
  // costs full waits for the loads in flight (the compiler cannot carry its count of
  // outstanding loads across two load sequences).
  // AMX: 0 every tile as stored, 1 every tile transposed, 2 tiles below t0 (2 <= t0 < nk) as
  // stored and the rest transposed, 3 tile 0 as stored and the rest transposed
  auto body = [&](auto AMC, int t0) {
    constexpr int AMX = decltype(AMC)::value;
    // A: lane l holds row mw + l % 32, k = 16 (l / 32) .. + 15 of each tile (a wave beyond M
    // loads row M - 1 and discards it, so that every wave issues the same loads)
    const int64_t arow_i = rows_ok ? mw + (lane & 31) : g.M - 1;
    const float* arow_t = (const float*)g.A + (kbeg + 16 * (lane >> 5)) * g.lda + arow_i;  // transposed
    const float* arow_d = (const float*)g.A + arow_i * g.lda + 16 * (lane >> 5) + kbeg;    // as stored
    float a0[16], a1[16], a2[16];
    auto loadA_t = [&](float (&a)[16], int t) {
      const float* src = arow_t + koff(t) * g.lda;
#pragma unroll
      for (int j = 0; j < 16; ++j) a[j] = src[j * g.lda];
    };
    auto loadA_d = [&](float (&a)[16], int t) {
      const float* src = arow_d + koff(t);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const f32x4 v = *((const f32x4*)(src + 4 * i));
        a[4 * i] = v[0];
        a[4 * i + 1] = v[1];
        a[4 * i + 2] = v[2];
        a[4 * i + 3] = v[3];
      }
    };
    // LM: the way tile t is read (0 as stored, 1 transposed), fixed at compile time
    auto loadA = [&](auto LM, float (&a)[16], int t) {
      if constexpr (decltype(LM)::value == 1) loadA_t(a, t);
      else loadA_d(a, t);
    };

    // B: load d of this wave covers stage bytes (wave * D + d) * 1024 + 16 * lane: piece and
    // first row uniform, the lane adding row lane / CHUNKS and its swizzled chunk.  In the
    // tile-major planes column n of the k tile at k0 starts at k0 ldb + 32 n.
    static_assert((1024 / ROWB) % (RPB * CHUNKS) == 0, "a load covers whole swizzle periods");
    static_assert(TL_BK == 32, "tile-major planes have 32-deep k tiles");
    const int rl = lane / CHUNKS, cs = (lane % CHUNKS) ^ ((rl / RPB) % CHUNKS);
    const uint32_t voff = (uint32_t)(rl * TL_BK + cs * 8);
    const __bf16* bbase[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int j = (wave * D + d) * 1024;
      const int p = j / PLB, r = (j % PLB) / ROWB;
      bbase[d] = (const __bf16*)g.B + p * g.b_plane + (n0 + r) * TL_BK + kbeg * g.ldb;
    }
    auto stage = [&](auto I) -> char* {
      constexpr int i = decltype(I)::value;
      if constexpr (i == 0) return st0;
      else if constexpr (i == 1) return st1;
      else return st2;
    };
    auto loadB = [&](auto I, int t) {
      char* dst = stage(I);
#pragma unroll
      for (int d = 0; d < D; ++d)
        __builtin_amdgcn_global_load_lds((const void*)(bbase[d] + koff(t) * g.ldb + voff),
                                         (lds_void*)(dst + (wave * D + d) * 1024), 16, 0, 0);
    };

    f32x16 acc[FN];
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;

    const int h = lane >> 5, cr = lane & 31;
    auto compute = [&](const char* S, const float (&a)[16]) {
      if (!rows_ok) return;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        float av[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) av[e] = a[8 * s + e];
        bf16x8 ap[NA];
        split_vec<NA>(av, ap);
        const int c = 2 * h + s;  // logical 16-byte chunk of k = 16 h + 8 s .. + 7
        // column blocks in pairs, the passes of the two alternating, so that no MFMA waits for
        // the one just before it (same accumulator)
#pragma unroll
        for (int b = 0; b < FN; b += 2) {
          bf16x8 bp[2][NB];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int r = (b + u) * 32 + cr;
#pragma unroll
            for (int p = 0; p < NB; ++p)
              bp[u][p] = *(const bf16x8*)(S + p * PLB + r * ROWB + ((c ^ ((r / RPB) % CHUNKS)) * 16));
          }
          // piece products smallest first
#pragma unroll
          for (int lvl = PMAX; lvl >= 0; --lvl)
#pragma unroll
            for (int pa = 0; pa < NA; ++pa) {
              const int pb = lvl - pa;
              if (pb < 0 || pb >= NB) continue;
#pragma unroll
              for (int u = 0; u < 2; ++u)
                acc[b + u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ap[pa], bp[u][pb], acc[b + u], 0, 0, 0);
            }
        }
      }
    };

    // tile t: B in stage t % 3, A in register set t % 3.  Iteration t issues the loads of tile
    // t + 2 (into the stage tile t - 1 used, released by the barrier that closed iteration
    // t - 1; past the last tile, the last tile again), computes tile t, then waits for tile
    // t + 1: at most the D + 4 loads of tile t + 2, issued after those of t + 1, may still be
    // outstanding.  Every wave issues the same loads in every iteration, so these counts are
    // exact and the compiler's own waits stay below them.
    // A loads per tile per wave: 4 as stored, 16 transposed
    const int tlast = nk - 1;
    auto wait_next = [&](auto LM) {  // LM: the way the tile whose loads went out last is read
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_waitcnt(tl_vmcnt(D + (decltype(LM)::value == 1 ? 16 : 4)));
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_waitcnt(tl_lgkm0());
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    };
    // LM: the way tile t + 2 is read
    auto step = [&](auto I, auto LM, float (&acur)[16], float (&anext2)[16], int t) {
      constexpr int i = decltype(I)::value;
      const int tn = t + 2 < tlast ? t + 2 : tlast;
      loadB(std::integral_constant<int, (i + 2) % 3>{}, tn);
      loadA(LM, anext2, tn);
      asm volatile("" ::: "memory");  // the loads of tile t + 2 go out before the MFMAs of tile t
      compute(stage(I), acur);
      wait_next(LM);
    };
    // iterations tb .. te - 1, the loads they issue all read the same way (stage and register
    // set of tile t are t % 3)
    auto run = [&](auto LM, int tb, int te) {
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, 1>;
      using I2 = std::integral_constant<int, 2>;
      int t = tb;
      if (t < te && t % 3 == 1) step(I1{}, LM, a1, a0, t++);
      if (t < te && t % 3 == 2) step(I2{}, LM, a2, a1, t++);
      for (; t + 3 <= te; t += 3) {
        step(I0{}, LM, a0, a2, t);
        step(I1{}, LM, a1, a0, t + 1);
        step(I2{}, LM, a2, a1, t + 2);
      }
      if (t < te) step(I0{}, LM, a0, a2, t++);
      if (t < te) step(I1{}, LM, a1, a0, t++);
    };

    const int t1 = nk > 1 ? 1 : 0;
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    if constexpr (AMX < 2) {
      using LM = std::integral_constant<int, AMX>;
      loadB(S0{}, 0);
      loadA(LM{}, a0, 0);
      loadB(S1{}, t1);
      loadA(LM{}, a1, t1);
      wait_next(LM{});  // tile 0
      run(LM{}, 0, nk);
    } else if constexpr (AMX == 2) {
      // (the choice of the way tile 1 is read is made at compile time too: a choice at run
      // time there costs the k loop full waits as well)
      loadB(S0{}, 0);
      loadA(S0{}, a0, 0);
      loadB(S1{}, t1);
      loadA(S0{}, a1, t1);
      wait_next(S0{});
      run(S0{}, 0, t0 - 2);  // tile t + 2 < t0
      run(S1{}, t0 - 2, nk);
    } else {
      loadB(S0{}, 0);
      loadA(S0{}, a0, 0);
      loadB(S1{}, t1);
      loadA(S1{}, a1, t1);
      wait_next(S1{});
      run(S1{}, 0, nk);
    }
    // no load may still be writing LDS or registers when the workgroup ends
    __builtin_amdgcn_s_waitcnt(tl_vmcnt(0));

    if (!rows_ok) return;
    // column-major partial sums: a lane holds rows 8 g + 4 h + j (j = 0..3) of column cr of
    // each 32-column block, one 16-byte store per g
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const uint32_t plr = (ln >> 5) * 4, plc = ln & 31;
    float* P = (float*)g.C + (int64_t)kc * g.M * g.N + n0 * g.M + mw;
    const uint32_t ldp = (uint32_t)g.M;
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
        *(float4*)(P + (b * 32 + plc) * ldp + q4 * 8 + plr) =
            make_float4(acc[b][4 * q4], acc[b][4 * q4 + 1], acc[b][4 * q4 + 2], acc[b][4 * q4 + 3]);
  };
  if constexpr (AM == 2) {
    // Rows m0 .. m0 + 255 span the 128-row tiles r = m0 / 128 and r + 1.  Columns below
    // (r + 1) 128 lie in lower or diagonal tiles for both and are read as stored; from
    // (r + 1) 128 on they lie in upper tiles, read transposed from the lower ones, except the
    // diagonal tile (r + 1, r + 1) of the second half, which is stored whole and exactly
    // symmetric and so is read transposed as well: one switch point for the workgroup.
    const int64_t ksw = (m0 / 128 + 1) * 128;
    // t0: the number of tiles of the chunk left of the switch column (k of tile t grows with t)
    int64_t t0l = 0;
    if (ksw > kbeg) {
      const int64_t u = (ksw - kbeg) / TL_BK, per = kper / TL_BK, run = 1 << lr;  // in tiles
      t0l = (u / per) * run + (u % per < run ? u % per : run);
    }
    const int t0 = (int)(t0l < nk ? t0l : nk);
    if (t0 == nk) body(std::integral_constant<int, 0>{}, nk);
    else if (t0 == 0) body(std::integral_constant<int, 1>{}, 0);
    else if (t0 >= 2) body(std::integral_constant<int, 2>{}, t0);
    else body(std::integral_constant<int, 3>{}, 1);
  } else {
    body(std::integral_constant<int, AM>{}, AM == 0 ? nk : 0);
  }
}

// Tile-major bf16 planes of a column-major panel: piece p of in[j * ldi + i] to
// out[p * rows * cols + (i / 32) * 32 cols + j * 32 + i % 32] (NP = 1: a bf16 panel copied)
template <int NP>
__global__ __launch_bounds__(256) void k_split_planes(const void* __restrict__ in, int64_t rows, int64_t cols,
                                                      int64_t ldi, __bf16* __restrict__ out) {
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4, j = blockIdx.y;
  if (i >= rows) return;
  __bf16 pc[4][NP];
  if constexpr (NP == 1) {
    const bf16x4 v = *(const bf16x4*)((const __bf16*)in + j * ldi + i);
#pragma unroll
    for (int e = 0; e < 4; ++e) pc[e][0] = v[e];
  } else {
    const f32x4 v = *(const f32x4*)((const float*)in + j * ldi + i);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (NP == 2) split2(v[e], pc[e][0], pc[e][1]);
      else split3(v[e], pc[e][0], pc[e][1], pc[e][2]);
    }
  }
  const int64_t o = (i / 32) * 32 * cols + j * 32 + i % 32;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    bf16x4 w = {pc[0][p], pc[1][p], pc[2][p], pc[3][p]};
    *(bf16x4*)(out + p * rows * cols + o) = w;
  }
}

template <int NA, int NB, int PMAX, int AM>
hipError_t launch_stream(const GemmArgs& g, int bn, int64_t blocks, hipStream_t s) {
  if (bn == 256) hipLaunchKernelGGL((k_tall_stream<256, NA, NB, PMAX, AM>), dim3((unsigned)blocks), dim3(512), 0, s, g);
  else hipLaunchKernelGGL((k_tall_stream<128, NA, NB, PMAX, AM>), dim3((unsigned)blocks), dim3(512), 0, s, g);
  return hipGetLastError();
}

}  // namespace

bool tall_stream_supported(const MixedGemm& mg) {
  const GemmArgs& g = mg.g;
  const bool kc = mg.a_kind == OK_F32_KC, mc = mg.a_kind == OK_F32_MC, sym = mg.a_kind == OK_F32_SYM;
  const bool combo = (kc && ((mg.na == 2 && mg.nb == 2 && mg.pmax == 1) || (mg.na == 3 && mg.nb == 1 && mg.pmax == 2) ||
                             (mg.na == 3 && mg.nb == 2 && mg.pmax == 2))) ||
                     (mc && ((mg.na == 2 && mg.nb == 3 && mg.pmax == 2) || (mg.na == 2 && mg.nb == 2 && mg.pmax == 1))) ||
                     (sym && mg.na == 2 && mg.nb == 2 && mg.pmax == 1 && g.M == g.K && g.M % 128 == 0);
  return combo && mg.b_kind == OK_BF16_KC && g.epi == EPI_COLSTORE && g.N % 128 == 0 &&
         g.M % 32 == 0 && g.M >= 1024 && g.splitk >= 1 && g.splitk <= 8 && 8 % g.splitk == 0 &&
         g.K % ((int64_t)TL_BK * g.splitk) == 0 && g.lda % 4 == 0 && g.b_tiled && g.ldb >= g.N &&
         g.b_plane % 8 == 0;
}

hipError_t tall_stream(const GemmArgs& run, const MixedGemm& mg, hipStream_t s) {
  const int bn = run.N % 256 == 0 ? 256 : 128;
  const int64_t MT = (run.M + TL_BM - 1) / TL_BM, NTT = run.N / bn, G = 8 / run.splitk;
  const int64_t blocks = 8 * ((MT + G - 1) / G) * NTT;  // row tiles beyond MT return at once
  if (mg.a_kind == OK_F32_SYM) return launch_stream<2, 2, 1, 2>(run, bn, blocks, s);
  if (mg.a_kind == OK_F32_MC) {
    if (mg.na == 2 && mg.nb == 3 && mg.pmax == 2) return launch_stream<2, 3, 2, 1>(run, bn, blocks, s);
    if (mg.na == 2 && mg.nb == 2 && mg.pmax == 1) return launch_stream<2, 2, 1, 1>(run, bn, blocks, s);
    return hipErrorInvalidValue;
  }
  if (mg.na == 2 && mg.nb == 2 && mg.pmax == 1) return launch_stream<2, 2, 1, 0>(run, bn, blocks, s);
  if (mg.na == 3 && mg.nb == 1 && mg.pmax == 2) return launch_stream<3, 1, 2, 0>(run, bn, blocks, s);
  if (mg.na == 3 && mg.nb == 2 && mg.pmax == 2) return launch_stream<3, 2, 2, 0>(run, bn, blocks, s);
  return hipErrorInvalidValue;
}

hipError_t split_planes(const void* in, int64_t rows, int64_t cols, int64_t ldi, int np, __bf16* out, hipStream_t s) {
  if (rows % 32 || ldi % 4 || rows > ldi || cols < 1 || cols > 65535 || np < 1 || np > 3) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((rows / 4 + 255) / 256), (unsigned)cols);
  if (np == 1) hipLaunchKernelGGL(k_split_planes<1>, grid, dim3(256), 0, s, in, rows, cols, ldi, out);
  else if (np == 2) hipLaunchKernelGGL(k_split_planes<2>, grid, dim3(256), 0, s, in, rows, cols, ldi, out);
  else hipLaunchKernelGGL(k_split_planes<3>, grid, dim3(256), 0, s, in, rows, cols, ldi, out);
  return hipGetLastError();
}

}  // namespace rb
