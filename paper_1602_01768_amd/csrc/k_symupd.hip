// Square updates on bf16 matrix cores.  Symmetric rank-2q update of the fixed-sketch
// step: X += c2 * [U W'] [W' U]^T on the lower BM x BM tiles of X (BM = 128 or 256), each
// tile also written to its mirrored position (the symmetric form of the update, eq. (qunac))
// -- or, when X is held on its lower 128 x 128 tiles only, written there alone (diagonal
// tiles whole); FULL: C += c2 * A B^T on every tile (the rank-q updates of AdaRBFGS,
// eq. (Cholimprov), and of the row variants of Alg. 1).
//
// Both operands are pre-split into two bf16 pieces (hi, lo), stored tile-major (each
// 32-column stage of a row tile contiguous, see pack_split2); the product keeps the
// piece products hi*hi + hi*lo + lo*hi with FP32 accumulation.  Unlike the general
// mixed GEMM, the operand tiles travel from memory straight into LDS
// (global_load_lds_dwordx4, 16 bytes per lane), so no registers stage them and no
// LDS stores sit between two barriers: the k loop is a ring of NS LDS stages of BKS
// columns each, with the loads of stage k + NS - 1 in flight while stage k is
// multiplied, and one barrier per stage.  Each stage lives in an LDS array of its
// own so that the compiler, which tracks these loads per LDS object, does not wait
// for the loads of later stages before reading an earlier one.
//
// LDS layout of a stage: [operand][piece][row][BKS bf16], rows unpadded, the 16-byte
// chunks of row r permuted by c ^ f(r) with f(r) = (r / (128 / row bytes)) % chunks,
// so that the eight lanes of a ds_read_b128 phase (eight consecutive rows, one chunk
// each) cover all 32 banks.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

// Launch shape, measured on the n = 16384, q = 256 update with random operands (same-run
// comparisons), for 128 x 128 tiles: two stages of 32 columns, two workgroups per CU and
// 2 x 2 waves of 64 x 64 were fastest; 16-column stages (any depth or occupancy), three or
// four stages (one workgroup per CU) and 2 x 1 / 1 x 2 wave grids were 10-40% slower, and an
// explicit interleave of LDS reads with MFMAs within 1%.  256 x 256 tiles halve the panel
// bytes per entry of X, which dominate the kernel's traffic (a tile reads 2 pieces of K
// columns of both panels, 8 K / BM bytes per entry of X against its 8 bytes read and
// written; without the panel loads the n = 16384, q = 256 update takes 0.33 ms instead of
// 0.64): two stages of 32 columns fill 128 KB of LDS, one workgroup of 2 x 4 waves of
// 128 x 64 per CU, which hides less of the load latency; the tile size is chosen per update
// by bf16_square_tile.
constexpr int UPD_BKS = 32;  // columns per stage
constexpr int UPD_NS = 2;    // stages in the ring
// The epilogue reads and writes X non-temporally when the panels are at least UPD_NT_MINQ
// columns wide: X passes once per launch while the bf16 panels are re-read by every tile,
// and streaming X past the caches keeps more of the panels in L2 (n = 16384, q = 256:
// 0.717 -> 0.671 ms; non-temporal stores alone 0.690 ms; n = 32768, q = 512: 4.50 -> 4.29 ms).
// With narrow panels the kernel only streams X, and there the non-temporal accesses cost
// write bandwidth (n = 32768, q = 32: 1.58 -> 2.20 ms).
constexpr int UPD_NT_MINQ = 128;

namespace rb {

namespace {

typedef __attribute__((address_space(3))) void lds_void;

RB_DEV void tri_index(int64_t t, int64_t& ti, int64_t& tj) {
  int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// s_waitcnt immediate for "at most n vector-memory operations outstanding" (gfx9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt and lgkmcnt left at their maxima)
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
// ... and for "no LDS operation outstanding" (lgkmcnt 0, vmcnt and expcnt at their maxima)
constexpr int lgkm0_imm() { return 15 | (3 << 14) | (7 << 4); }

// NP: bf16 pieces per operand, 2 (products hi*hi, hi*lo, lo*hi) or 3 (the six products of total
// weight >= 2^-16, every FP32 entry represented exactly)
template <int BM, int BKS, int NS, int OCC, int WAVES_M, int WAVES_N, bool FULL, int NTX, bool MIRROR = true,
          int NP = 2>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) __attribute__((amdgpu_waves_per_eu(OCC * WAVES_M * WAVES_N / 4, 8)))
void k_symupd_dma(GemmArgs g) {
  constexpr int NW = WAVES_M * WAVES_N;
  static_assert(NP == 2 || NP == 3, "pieces");
  constexpr int WM = BM / WAVES_M, WN = BM / WAVES_N, FM = WM / 32, FN = WN / 32;
  constexpr int ROWB = BKS * 2;                 // bytes of one row of one piece
  constexpr int CHUNKS = ROWB / 16;             // 16-byte chunks per row
  constexpr int RPB = 128 / ROWB;               // rows per 128-byte bank period
  constexpr int PLB = BM * ROWB;                // bytes of one piece of one operand
  constexpr int OPB = NP * PLB;                 // bytes of one operand
  constexpr int STB = 2 * OPB;                  // bytes of one stage
  constexpr int D = STB / 1024 / NW;            // 1 KB loads per wave per stage
  static_assert(BKS == 16 || BKS == 32 || BKS == 64, "stage depth");
  static_assert(BM == 128 || BM == 256, "tile edge");
  static_assert(NS >= 2 && NS <= 4, "stages");
  __shared__ __attribute__((aligned(1024))) char st0[STB];
  __shared__ __attribute__((aligned(1024))) char st1[STB];
  __shared__ __attribute__((aligned(1024))) char st2[NS > 2 ? STB : 16];
  __shared__ __attribute__((aligned(1024))) char st3[NS > 3 ? STB : 16];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;

  // tile of this workgroup: each XCD (blockIdx % 8) takes a contiguous run of the order
  const int64_t T = g.M / BM;
  const int64_t NTT = g.tiles ? g.ntiles : (FULL ? T * T : T * (T + 1) / 2);
  const int64_t per = (NTT + 7) / 8, t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= NTT) return;
  int64_t mt, nt;
  if (g.tiles) {
    mt = g.tiles[t].x;
    nt = g.tiles[t].y;
  } else if (FULL) {
    mt = t / T;
    nt = t % T;
  } else {
    tri_index(t, mt, nt);
  }
  const bool diag = !FULL && mt == nt;
  const int64_t m0 = mt * BM, n0 = nt * BM;

  // Sources of this wave's D loads per stage: load d covers stage bytes
  // (wave * D + d) * 1024 + 16 * lane, i.e. operand, piece and first row are uniform
  // across the wave (a scalar base), and the lane adds row lane / CHUNKS and its
  // swizzled chunk -- the same for every d, as each load covers a multiple of the
  // swizzle period of rows (a 32-bit vector offset per operand).
  // The panels are stored tile-major (pack_split2 with tile = BM): a stage of a row tile is
  // BM x 32 contiguous, so each load reads 1 KB of whole 128-byte lines (row-major panels give
  // each load 16 half lines, the other halves read again by the next stage), and the stage of
  // k0 starts k0 BM entries into the row tile's block of BM x ld entries.
  static_assert((1024 / ROWB) % (RPB * CHUNKS) == 0, "a load covers whole swizzle periods");
  static_assert(BKS == 32, "tile-major panels have 32-column stages");
  const int rl = lane / CHUNKS, cs = (lane % CHUNKS) ^ ((rl / RPB) % CHUNKS);
  const uint32_t voff = (uint32_t)(rl * BKS + cs * 8);
  const __bf16* ubase[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int j = (wave * D + d) * 1024;
    const int o = j / OPB, p = (j % OPB) / PLB, r = (j % PLB) / ROWB;
    ubase[d] = o == 0 ? (const __bf16*)g.A + p * g.a_plane + m0 * g.lda + r * BKS
                      : (const __bf16*)g.B + p * g.b_plane + n0 * g.ldb + r * BKS;
  }
  auto stage = [&](auto I) -> char* {
    constexpr int i = decltype(I)::value;
    if constexpr (i == 0) return st0;
    else if constexpr (i == 1) return st1;
    else if constexpr (i == 2) return st2;
    else return st3;
  };
  auto issue = [&](auto I, int64_t k0) {
    char* dst = stage(I);
#pragma unroll
    for (int d = 0; d < D; ++d)
      __builtin_amdgcn_global_load_lds((const void*)(ubase[d] + k0 * BM + voff),
                                       (lds_void*)(dst + (wave * D + d) * 1024), 16, 0, 0);
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  // byte offset of this lane's fragment row within a piece, and its chunk swizzle
  const int ra = wm * WM + (lane & 31), rb = wn * WN + (lane & 31);
  auto compute = [&](const char* S) {
#pragma unroll
    for (int s = 0; s < BKS / 16; ++s) {
      const int c = 2 * s + (lane >> 5);
      bf16x8 av[NP][FM], bv[NP][FN];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int a = 0; a < FM; ++a) {
          const int r = ra + a * 32;
          av[p][a] = *(const bf16x8*)(S + p * PLB + r * ROWB + ((c ^ ((r / RPB) % CHUNKS)) * 16));
        }
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          const int r = rb + b * 32;
          bv[p][b] = *(const bf16x8*)(S + OPB + p * PLB + r * ROWB + ((c ^ ((r / RPB) % CHUNKS)) * 16));
        }
      // piece products smallest first (pa + pb = NP - 1 down to 0)
#pragma unroll
      for (int lvl = NP - 1; lvl >= 0; --lvl)
#pragma unroll
        for (int pa = 0; pa < NP; ++pa) {
          const int pb = lvl - pa;
          if (pb < 0 || pb >= NP) continue;
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[pa][a], bv[pb][b], acc[a][b], 0, 0, 0);
        }
    }
  };

  // Old values of this wave's 32 x 32 output blocks, read two blocks ahead.  Offsets
  // are 32-bit from the wave's block origin (a uniform base), and the lane index the
  // epilogue derives them from is made opaque after the k loop, so that the compiler
  // computes the epilogue addresses there instead of holding them through the loop.
  const uint32_t ld = (uint32_t)g.ldc;
  float* Xd = (float*)g.C + (m0 + wm * WM) * g.ldc + (n0 + wn * WN);
  float* Xm = (float*)g.C + (n0 + wn * WN) * g.ldc + (m0 + wm * WM);
  float oldv[2][16];
  auto load_old = [&](int i, float (&o)[16], int ln) {
    const int a = i / FN, b = i % FN;
    const uint32_t lr = (ln >> 5) * 4, lc = ln & 31;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float* src = Xd + (a * 32 + (r >> 2) * 8 + lr + (r & 3)) * ld + b * 32 + lc;
      if constexpr (NTX == 1) o[r] = __builtin_nontemporal_load(src);
      else o[r] = *src;
    }
  };
  load_old(0, oldv[0], lane);
  load_old(1, oldv[1], lane);

  // k loop: step k uses stage k % NS; the loads of step k + NS - 1 go into the stage
  // that step k - 1 used, which the barrier of step k has released
  const int nk = (int)(g.K / BKS);
  if (nk > 0) issue(std::integral_constant<int, 0>{}, 0);
  if constexpr (NS > 2)
    if (nk > 1) issue(std::integral_constant<int, 1>{}, (int64_t)BKS);
  if constexpr (NS > 3)
    if (nk > 2) issue(std::integral_constant<int, 2>{}, (int64_t)2 * BKS);
  auto step = [&](auto I, int k) {
    constexpr int i = decltype(I)::value;
    if (k >= nk) return;
    // this wave's loads of step k are complete once at most the loads issued after
    // them are outstanding: those of steps k + 1 .. k + NS - 2 (D each), and with the
    // L2 touch the D dwords of the touch issued right after them (if there was one)
    asm volatile("" ::: "memory");  // the loads counted here stay above the wait
    if (k + NS - 2 < nk) __builtin_amdgcn_s_waitcnt(vmcnt_imm((NS - 2) * D));
    else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    // LDS-only barrier: every wave has its loads of step k in LDS (waited above) and has
    // finished reading stage k - 1 (lgkmcnt); no global-memory ordering is needed here,
    // so the workgroup fence of __syncthreads (which would also wait for the loads in
    // flight) is left out.  The empty asm statements keep the compiler from moving LDS
    // accesses across it.
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(lgkm0_imm());
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (k + NS - 1 < nk) issue(std::integral_constant<int, (i + NS - 1) % NS>{}, (int64_t)(k + NS - 1) * BKS);
    compute(stage(I));
  };
  for (int kb = 0; kb < nk; kb += NS) {
    step(std::integral_constant<int, 0>{}, kb);
    step(std::integral_constant<int, 1>{}, kb + 1);
    if constexpr (NS > 2) step(std::integral_constant<int, 2 % NS>{}, kb + 2);
    if constexpr (NS > 3) step(std::integral_constant<int, 3 % NS>{}, kb + 3);
  }

  // X += c2 * acc one 32 x 32 block at a time.  A lane holds column lc and rows
  // 8 g + lr + j (j = 0..3) of the block: the same values are row lc, four
  // consecutive columns, of the mirrored block, written as one 16-byte store per g.
  const float c2 = (float)g.c2;
  int ln = lane;
  asm volatile("" : "+v"(ln));
  const uint32_t lr = (ln >> 5) * 4, lc = ln & 31;
  const int dofs = (int)((m0 + wm * WM) - (n0 + wn * WN));
  constexpr int NBLK = FM * FN;
#pragma unroll
  for (int i = 0; i < NBLK; ++i) {
    const int a = i / FN, b = i % FN;
    float nvs[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) nvs[r] = oldv[i & 1][r] + c2 * acc[a][b][r];
    if (i + 2 < NBLK) load_old(i + 2, oldv[i & 1], ln);
    if (!diag) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float* dst = Xd + (a * 32 + (r >> 2) * 8 + lr + (r & 3)) * ld + b * 32 + lc;
        if constexpr (NTX != 0) __builtin_nontemporal_store(nvs[r], dst);
        else *dst = nvs[r];
      }
      if constexpr (!FULL && MIRROR) {
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          typedef float f32x4v __attribute__((ext_vector_type(4)));
          f32x4v* dst = (f32x4v*)(Xm + (b * 32 + lc) * ld + a * 32 + 8 * q4 + lr);
          const f32x4v v = {nvs[4 * q4], nvs[4 * q4 + 1], nvs[4 * q4 + 2], nvs[4 * q4 + 3]};
          if constexpr (NTX != 0) __builtin_nontemporal_store(v, dst);
          else *dst = v;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t ml = (r >> 2) * 8 + lr + (r & 3);
        const int dd = dofs + a * 32 + (int)ml - b * 32 - (int)lc;  // m - n of this element
        if (dd >= 0) Xd[(a * 32 + ml) * ld + b * 32 + lc] = nvs[r];
        if (dd > 0) Xm[(b * 32 + lc) * ld + a * 32 + ml] = nvs[r];
      }
    }
  }
}

}  // namespace

namespace {

template <int BM, int OCC, int WM, int WN>
hipError_t launch_symupd(const GemmArgs& g, int64_t blocks, hipStream_t s) {
  const dim3 grid((unsigned)blocks), block(64 * WM * WN);
  const bool full = g.epi == EPI_ADDROW;
  const bool nt = (full ? g.K : g.K / 2) >= UPD_NT_MINQ;  // panel width q
  if (full && nt)
    hipLaunchKernelGGL((k_symupd_dma<BM, UPD_BKS, UPD_NS, OCC, WM, WN, true, 1>), grid, block, 0, s, g);
  else if (full)
    hipLaunchKernelGGL((k_symupd_dma<BM, UPD_BKS, UPD_NS, OCC, WM, WN, true, 0>), grid, block, 0, s, g);
  else if (g.lower_only && nt)
    hipLaunchKernelGGL((k_symupd_dma<BM, UPD_BKS, UPD_NS, OCC, WM, WN, false, 1, false>), grid, block, 0, s, g);
  else if (g.lower_only)
    hipLaunchKernelGGL((k_symupd_dma<BM, UPD_BKS, UPD_NS, OCC, WM, WN, false, 0, false>), grid, block, 0, s, g);
  else if (nt)
    hipLaunchKernelGGL((k_symupd_dma<BM, UPD_BKS, UPD_NS, OCC, WM, WN, false, 1>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((k_symupd_dma<BM, UPD_BKS, UPD_NS, OCC, WM, WN, false, 0>), grid, block, 0, s, g);
  return hipGetLastError();
}

// Symmetric update with 3 pieces per operand (128 x 128 tiles; two 48 KB stages, one workgroup
// of 2 x 2 waves per CU)
hipError_t launch_symupd3(const GemmArgs& g, int64_t blocks, hipStream_t s) {
  const dim3 grid((unsigned)blocks), block(256);
  const bool nt = g.K / 2 >= UPD_NT_MINQ;
  if (g.lower_only && nt)
    hipLaunchKernelGGL((k_symupd_dma<128, UPD_BKS, UPD_NS, 1, 2, 2, false, 1, false, 3>), grid, block, 0, s, g);
  else if (g.lower_only)
    hipLaunchKernelGGL((k_symupd_dma<128, UPD_BKS, UPD_NS, 1, 2, 2, false, 0, false, 3>), grid, block, 0, s, g);
  else if (nt)
    hipLaunchKernelGGL((k_symupd_dma<128, UPD_BKS, UPD_NS, 1, 2, 2, false, 1, true, 3>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((k_symupd_dma<128, UPD_BKS, UPD_NS, 1, 2, 2, false, 0, true, 3>), grid, block, 0, s, g);
  return hipGetLastError();
}

}  // namespace

// g.bn: the tile edge (256, or 128 for any other value), as bf16_square_tile gives it;
// g.upd_pieces: 2, or 3 (symmetric update on 128 x 128 tiles only)
hipError_t symupd_bf16_dma(const GemmArgs& g, int64_t blocks, hipStream_t s) {
  const int bm = g.bn == 256 ? 256 : 128;
  if (g.K % UPD_BKS || g.M % bm || g.M != g.N || g.lda % 8 || g.ldb % 8 || g.a_plane % 8 || g.b_plane % 8 ||
      g.ldc % 4 || (g.upd_pieces != 2 && g.upd_pieces != 3) ||
      (g.upd_pieces == 3 && (bm != 128 || g.epi != EPI_SYMUPD)))
    return hipErrorInvalidValue;
  if (g.upd_pieces == 3) return launch_symupd3(g, blocks, s);
  if (bm == 256) return launch_symupd<256, 1, 2, 4>(g, blocks, s);
  return launch_symupd<128, 2, 2, 2>(g, blocks, s);
}

namespace {

// One workgroup per strictly lower 128 x 128 tile (ti, tj), tj < ti, numbered row by row;
// its sixteen 32 x 32 blocks go through a padded LDS transpose onto tile (tj, ti).
__global__ __launch_bounds__(256) void k_mirror_lower(float* X, int64_t ld) {
  __shared__ float tb[32][33];
  const int64_t b = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * (double)b + 1.0) + 1.0) * 0.5);
  while (ti * (ti - 1) / 2 > b) --ti;
  while ((ti + 1) * ti / 2 <= b) ++ti;
  const int64_t tj = b - ti * (ti - 1) / 2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int bi = 0; bi < 4; ++bi)
    for (int bj = 0; bj < 4; ++bj) {
      const int64_t r0 = ti * 128 + bi * 32, c0 = tj * 128 + bj * 32;
      __syncthreads();
      for (int y = ty; y < 32; y += 8) tb[y][tx] = X[(r0 + y) * ld + c0 + tx];
      __syncthreads();
      for (int y = ty; y < 32; y += 8) X[(c0 + y) * ld + r0 + tx] = tb[tx][y];
    }
}

}  // namespace

hipError_t mirror_lower(float* X, int64_t ld, int64_t T, hipStream_t s) {
  const int64_t nb = T * (T - 1) / 2;
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mirror_lower, dim3((unsigned)nb), dim3(256), 0, s, X, ld);
  return hipGetLastError();
}

}  // namespace rb
