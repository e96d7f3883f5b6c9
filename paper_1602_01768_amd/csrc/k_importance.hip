// Importance weights for simultaneous randomized Kaczmarz over the partition into
// consecutive blocks C_b of q coordinates (eq. discoptprob with W = I and X_k in place of
// A^-1): w_b^2 = ||X_k I_{:C_b} I_{C_b:} A||_F^2 = <(Z Z^T)_{C_b C_b}, (A A^T)_{C_b C_b}>
// with Z = X_k^T.  All blocks are formed in one launch: a workgroup takes one block b, one
// lower TW x TW tile (ti >= tj) of its q x q Gram and one chunk of the n-long sum, runs
// v_mfma_f64_16x16x4f64 over it, and dots its tile with the matching tile of (A A^T)_{C_b C_b}
// in the epilogue (off-diagonal tiles twice, both Gram blocks being symmetric), so that no
// Gram matrix is stored.  A second kernel sums the partials of each block in a fixed order.
#include <algorithm>

#include "common.hpp"
#include "importance.hpp"
#include "kernels.hpp"

namespace rb {

namespace {

constexpr int IW_BK = 32;  // k depth of one LDS stage

struct WeightPlan {
  int tw = 64, nt = 1, ks = 1;
  int64_t r = 0, kchunk = IW_BK;
};

// Tile width 64 (2 x 2 waves of 32 x 32) for q > 32, else 32 (waves of 16 x 16); the sum over
// k is split so that the launch has about 2048 workgroups, each chunk at least 256 deep.
WeightPlan weight_plan(int64_t n, int q) {
  WeightPlan p;
  p.tw = q > 32 ? 64 : 32;
  const int T = (q + p.tw - 1) / p.tw;
  p.nt = T * (T + 1) / 2;
  p.r = n / q;
  const int64_t tiles = p.r * p.nt;
  int64_t ks = (2048 + tiles - 1) / tiles;
  ks = std::max<int64_t>(1, std::min<int64_t>(ks, n / 256));
  int64_t kc = (n + ks - 1) / ks;
  kc = (kc + IW_BK - 1) / IW_BK * IW_BK;
  p.kchunk = std::max<int64_t>(kc, IW_BK);
  p.ks = (int)((n + p.kchunk - 1) / p.kchunk);
  return p;
}

// EPT consecutive entries p[k .. k + EPT) as doubles; entries at or past kend read as 0.
// full: all of them are below kend and p + k is 16-byte aligned.
template <class T, int EPT>
RB_DEV void load_run(const T* p, int64_t k, int64_t kend, bool full, double* out) {
  if (full) {
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int e = 0; e < EPT; e += 4) {
        const float4 v = *(const float4*)(p + k + e);
        out[e] = v.x;
        out[e + 1] = v.y;
        out[e + 2] = v.z;
        out[e + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT; e += 2) {
        const double2 v = *(const double2*)(p + k + e);
        out[e] = v.x;
        out[e + 1] = v.y;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < EPT; ++e) out[e] = (k + e < kend) ? (double)p[k + e] : 0.0;
  }
}

RB_DEV void tri_pair(int t, int& ti, int& tj) {
  ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  tj = t - ti * (ti + 1) / 2;
}

// One workgroup: block b, lower tile (ti, tj), k chunk kc; part[x] = the tile's share of
// <P_b P_b^T, Q_b> over the chunk (x = (b nt + tile) ks + kc).
template <class T, int TW>
__global__ __launch_bounds__(256) void k_block_gram_dot(const T* P, int64_t ld, int64_t n, int q, const double* Q,
                                                        int64_t qld, int nt, int ks, int64_t kchunk, bool vec,
                                                        double* part) {
  constexpr int BK = IW_BK, WT = TW / 2, F = WT / 16;
  constexpr int EPT = TW * BK / 256, TPC = BK / EPT;  // entries per thread, threads per vector
  static_assert(EPT % 4 == 0, "vector loads take 4 entries");
  __shared__ double As[BK * (TW + 1)];
  __shared__ double Bs[BK * (TW + 1)];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t x = blockIdx.x;
  const int kc = (int)(x % ks);
  const int tile = (int)((x / ks) % nt);
  const int64_t b = x / ((int64_t)ks * nt);
  int ti, tj;
  tri_pair(tile, ti, tj);
  const bool diag = ti == tj;
  const int64_t kbeg = (int64_t)kc * kchunk;
  const int64_t kend = min(n, kbeg + kchunk);
  const int lm = tid / TPC, lk = (tid % TPC) * EPT;
  const int ca = ti * TW + lm, cb = tj * TW + lm;  // block-local vectors this thread stages
  const T* pa = ca < q ? P + (b * q + ca) * ld : nullptr;
  const T* pb = cb < q ? P + (b * q + cb) * ld : nullptr;
  const double* Bsrc = diag ? As : Bs;

  double ra[EPT], rbv[EPT];
  auto gload = [&](int64_t k0) {
    const bool full = vec && k0 + BK <= kend;
    if (pa) load_run<T, EPT>(pa, k0 + lk, kend, full, ra);
    else
#pragma unroll
      for (int e = 0; e < EPT; ++e) ra[e] = 0.0;
    if (!diag) {
      if (pb) load_run<T, EPT>(pb, k0 + lk, kend, full, rbv);
      else
#pragma unroll
        for (int e = 0; e < EPT; ++e) rbv[e] = 0.0;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int e = 0; e < EPT; ++e) As[(lk + e) * (TW + 1) + lm] = ra[e];
    if (!diag)
#pragma unroll
      for (int e = 0; e < EPT; ++e) Bs[(lk + e) * (TW + 1) + lm] = rbv[e];
  };

  f64x4 acc[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int c = 0; c < F; ++c) acc[a][c] = (f64x4){0.0, 0.0, 0.0, 0.0};

  if (kbeg < kend) gload(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + BK < kend) gload(k0 + BK);
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      // lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16) of the 16 x 4 x 16 step
      const int kr = k4 * 4 + (lane >> 4);
      double av[F], bv[F];
#pragma unroll
      for (int a = 0; a < F; ++a) av[a] = As[kr * (TW + 1) + wm * WT + a * 16 + (lane & 15)];
#pragma unroll
      for (int c = 0; c < F; ++c) bv[c] = Bsrc[kr * (TW + 1) + wn * WT + c * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < F; ++a)
#pragma unroll
        for (int c = 0; c < F; ++c) acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
    }
  }

  // lane l holds Gram entries (row l / 16 + 4 r, column l % 16) of each 16 x 16 block
  const int lr = lane >> 4, lc = lane & 15;
  const double* Qb = Q + b * qld * qld;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int c = 0; c < F; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = ti * TW + wm * WT + a * 16 + lr + 4 * r, cc = tj * TW + wn * WT + c * 16 + lc;
        if (m < q && cc < q) s = fma(acc[a][c][r], Qb[m + cc * qld], s);
      }
  if (!diag) s *= 2.0;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (tid == 0) part[x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// t[j] for j = b q: the square root of the block's partials summed in index order; other j: 0.
__global__ __launch_bounds__(256) void k_block_weights_finish(const double* part, int per, int64_t n, int q,
                                                              double* t) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  if (j % q) {
    t[j] = 0.0;
    return;
  }
  const double* p = part + (j / q) * per;
  double v = 0.0;
  for (int i = 0; i < per; ++i) v += p[i];
  t[j] = v > 0.0 ? sqrt(v) : 0.0;
}

}  // namespace

int64_t block_weights_workspace(int64_t n, int q) {
  if (q < 1 || n < q) return 0;
  const WeightPlan p = weight_plan(n, q);
  return p.r * p.nt * p.ks;
}

hipError_t block_gram_weights(const void* P, int dt, int64_t ld, int64_t n, int q, const double* Q, int64_t qld,
                              double* part, int64_t part_cap, double* t, hipStream_t s) {
  if (!P || !Q || !part || !t || q < 1 || n < q || n % q || qld < q || ld < n || (dt != DT_F32 && dt != DT_F64))
    return hipErrorInvalidValue;
  const WeightPlan p = weight_plan(n, q);
  const int64_t blocks = p.r * p.nt * p.ks;
  if (blocks > part_cap || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const bool vec = ld % 4 == 0 && ((uintptr_t)P & 15) == 0;
  const dim3 grid((unsigned)blocks), blk(256);
  if (dt == DT_F32) {
    if (p.tw == 64)
      hipLaunchKernelGGL((k_block_gram_dot<float, 64>), grid, blk, 0, s, (const float*)P, ld, n, q, Q, qld, p.nt, p.ks,
                         p.kchunk, vec, part);
    else
      hipLaunchKernelGGL((k_block_gram_dot<float, 32>), grid, blk, 0, s, (const float*)P, ld, n, q, Q, qld, p.nt, p.ks,
                         p.kchunk, vec, part);
  } else {
    if (p.tw == 64)
      hipLaunchKernelGGL((k_block_gram_dot<double, 64>), grid, blk, 0, s, (const double*)P, ld, n, q, Q, qld, p.nt,
                         p.ks, p.kchunk, vec, part);
    else
      hipLaunchKernelGGL((k_block_gram_dot<double, 32>), grid, blk, 0, s, (const double*)P, ld, n, q, Q, qld, p.nt,
                         p.ks, p.kchunk, vec, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_block_weights_finish, dim3((unsigned)ceil_div(n, 256)), blk, 0, s, part, p.nt * p.ks, n, q, t);
  return hipGetLastError();
}

}  // namespace rb
