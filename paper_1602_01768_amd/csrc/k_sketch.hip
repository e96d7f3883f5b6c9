// Sketch generation on the device from the counter-based stream (see rbfgs.h):
// Gaussian sketches (Box-Muller on Philox4x64-10 words, rounded to bf16 values)
// and coordinate sketches (Floyd's sampling with Lemire's bounded draws).
#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace rb {

__global__ void k_sketch_gauss(uint64_t seed, uint64_t k, const int64_t* kbase, int64_t n, int64_t q, void* S, int dt,
                               int64_t ld) {
  if (kbase) k += (uint64_t)*kbase;  // iteration = device counter + offset (replayed graphs)
  const int64_t total = n * q;
  const int64_t nblocks = (total + 3) / 4;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblocks; b += (int64_t)gridDim.x * blockDim.x) {
    const u64x4 w = philox4x64_10((uint64_t)b, k, KIND_GAUSS, 0, seed, 0);
#pragma unroll
    for (int word = 0; word < 4; ++word) {
      const int64_t e = 4 * b + word;
      if (e >= total) break;
      const double z = gauss_entry_from_block(w, word);
      const int64_t i = e % n, j = e / n;
      const int64_t idx = i + j * ld;
      if (dt == DT_F64) ((double*)S)[idx] = z;
      else if (dt == DT_F32) ((float*)S)[idx] = (float)z;
      else ((__bf16*)S)[idx] = (__bf16)(float)z;  // z is already a bf16 value: exact
    }
  }
}

hipError_t sketch_gauss(uint64_t seed, int64_t k, int64_t n, int32_t q, void* S, int dt, int64_t ld, hipStream_t s,
                        const int64_t* kbase) {
  const int64_t nblocks = (n * (int64_t)q + 3) / 4;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(nblocks, 256), 4096));
  hipLaunchKernelGGL(k_sketch_gauss, dim3(grid), dim3(256), 0, s, seed, (uint64_t)k, kbase, n, (int64_t)q, S, dt, ld);
  return hipGetLastError();
}

__global__ void k_add_i64(int64_t* c, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c += v;
}

hipError_t add_i64(int64_t* c, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(64), 0, s, c, v);
  return hipGetLastError();
}

// Sequential reader of the 64-bit words of one iteration's coordinate stream.
struct WordStream {
  uint64_t seed, k, pos, block;
  u64x4 w;
  RB_DEV uint64_t next() {
    const uint64_t b = pos >> 2;
    if (b != block) {
      w = philox4x64_10(b, k, KIND_COORD, 0, seed, 0);
      block = b;
    }
    const int i = (int)(pos & 3);
    ++pos;
    return i == 0 ? w.x : (i == 1 ? w.y : (i == 2 ? w.z : w.w));
  }
  // Uniform integer in [0, m), m >= 1: Lemire's multiply with rejection.
  RB_DEV uint64_t bounded(uint64_t m) {
    uint64_t x = next();
    uint64_t lo = x * m;
    if (lo < m) {
      const uint64_t thresh = (0ull - m) % m;
      while (lo < thresh) {
        x = next();
        lo = x * m;
      }
    }
    return __umul64hi(x, m);
  }
};

// One workgroup: Floyd's algorithm on thread 0 over a bitmap of [0, n) in LDS,
// then a block-wide scan of the bitmap writes the chosen indices in ascending order.
__global__ __launch_bounds__(256) void k_sketch_coord(uint64_t seed, uint64_t k, int64_t n, int q, int32_t* idx) {
  extern __shared__ uint32_t bits[];
  __shared__ int counts[256];
  const int nwords = (int)((n + 31) / 32);
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) bits[i] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    WordStream st{seed, k, 0ull, ~0ull, {0, 0, 0, 0}};
    for (int64_t j = n - q; j < n; ++j) {
      const int64_t t = (int64_t)st.bounded((uint64_t)(j + 1));
      const uint32_t tb = 1u << (t & 31);
      const int64_t pick = (bits[t >> 5] & tb) ? j : t;
      bits[pick >> 5] |= 1u << (pick & 31);
    }
  }
  __syncthreads();
  const int per = (nwords + 255) / 256;
  const int w0 = threadIdx.x * per, w1 = min(nwords, w0 + per);
  int c = 0;
  for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
  counts[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < 256; ++i) {
      const int v = counts[i];
      counts[i] = run;
      run += v;
    }
  }
  __syncthreads();
  int out = counts[threadIdx.x];
  for (int w = w0; w < w1; ++w) {
    uint32_t m = bits[w];
    while (m) {
      const int b = __ffs(m) - 1;
      m &= m - 1;
      idx[out++] = w * 32 + b;
    }
  }
}

hipError_t sketch_coord(uint64_t seed, int64_t k, int64_t n, int32_t q, int32_t* idx, hipStream_t s) {
  const size_t lds = sizeof(uint32_t) * (size_t)((n + 31) / 32);
  static std::once_flag once;  // contexts may be driven from several host threads
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute((const void*)k_sketch_coord, hipFuncAttributeMaxDynamicSharedMemorySize, 131072);
  });
  if (attr_err != hipSuccess) return attr_err;
  hipLaunchKernelGGL(k_sketch_coord, dim3(1), dim3(256), lds, s, seed, (uint64_t)k, n, (int)q, idx);
  return hipGetLastError();
}


// Partition sampling (the probabilities of eq. ihsih0 over consecutive blocks
// C_i = [i q, (i+1) q), q dividing n): block weight w_i = max(0, sum_{j in C_i} t_j);
// block i is the first whose running weight sum exceeds u times the total,
// u = ((x >> 11) + 0.5) 2^-53 from word 0 of block 0 of iteration k's stream (kind 3);
// if rounding leaves no crossing, the last block with positive weight is drawn.  Writes
// idx[0..q) = C_i and ht = total / w_i, the Horvitz-Thompson factor 1/p_i.  A total that
// is not finite and positive sets status 4 and draws block 0.  One workgroup, two forms:
//  * q >= 64 and at most SAMPLE_LDS blocks: one wave per block (lanes stride the block,
//    a fixed shuffle tree adds them) into LDS, then thread 0 scans the block weights;
//  * otherwise each thread sums a contiguous run of whole blocks, thread 0 scans the run
//    totals, and the thread whose run holds the crossing scans it again.
constexpr int SAMPLE_LDS = 4096;

__global__ __launch_bounds__(256) void k_sample_partition(const double* t, int64_t n, int q, uint64_t seed, uint64_t k,
                                                          int32_t* idx, double* ht, int* status) {
  __shared__ double wl[SAMPLE_LDS];
  __shared__ double run[256];
  __shared__ double sh_thr, sh_before, sh_total;
  __shared__ int sh_owner;
  __shared__ int64_t sh_pick;
  const int64_t r = n / q;
  auto weight = [&](int64_t b) {
    double w = 0.0;
    for (int64_t j = b * q; j < (b + 1) * q; ++j) w += t[j];
    return w > 0.0 ? w : 0.0;
  };
  const u64x4 words = philox4x64_10(0, k, KIND_PART, 0, seed, 0);
  const double u = ((double)(words.x >> 11) + 0.5) * 0x1.0p-53;
  if (q >= 64 && r <= SAMPLE_LDS) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t b = wave; b < r; b += 4) {
      double v = 0.0;
      for (int j = lane; j < q; j += 64) v += t[b * q + j];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) wl[b] = v > 0.0 ? v : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double total = 0.0;
      for (int64_t b = 0; b < r; ++b) total += wl[b];
      const double thr = u * total;
      int64_t pick = -1, last = 0;
      double c = 0.0;
      for (int64_t b = 0; b < r; ++b) {
        if (!(wl[b] > 0.0)) continue;
        last = b;
        c += wl[b];
        if (c > thr) {
          pick = b;
          break;
        }
      }
      if (pick < 0) pick = last;
      const bool ok = total > 0.0 && isfinite(total);
      if (!ok) {
        pick = 0;
        if (status) atomicCAS(status, 0, 4);
      }
      sh_pick = pick;
      if (ht) ht[0] = ok ? total / wl[pick] : 1.0;
    }
    __syncthreads();
  } else {
    const int64_t per = (r + 255) / 256;
    const int64_t b0 = min<int64_t>(r, (int64_t)threadIdx.x * per), b1 = min<int64_t>(r, b0 + per);
    double mine = 0.0;
    for (int64_t b = b0; b < b1; ++b) mine += weight(b);
    run[threadIdx.x] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
      double total = 0.0;
      for (int i = 0; i < 256; ++i) total += run[i];
      const double thr = u * total;
      int owner = -1, last = -1;
      double c = 0.0, before = 0.0, before_last = 0.0;
      for (int i = 0; i < 256; ++i) {
        if (!(run[i] > 0.0)) continue;
        if (c + run[i] > thr) {
          owner = i;
          before = c;
          break;
        }
        last = i;
        before_last = c;
        c += run[i];
      }
      if (owner < 0) {
        owner = last;
        before = before_last;
      }
      if (!(total > 0.0) || !isfinite(total)) {
        owner = -1;
        if (status) atomicCAS(status, 0, 4);
      }
      sh_owner = owner;
      sh_thr = thr;
      sh_before = before;
      sh_total = total;
      sh_pick = 0;
    }
    __syncthreads();
    if ((int)threadIdx.x == sh_owner) {
      double c = sh_before;
      int64_t pick = -1, last = b0;
      for (int64_t b = b0; b < b1; ++b) {
        const double w = weight(b);
        if (!(w > 0.0)) continue;
        last = b;
        c += w;
        if (c > sh_thr) {
          pick = b;
          break;
        }
      }
      pick = pick >= 0 ? pick : last;
      sh_pick = pick;
      if (ht) ht[0] = sh_total / weight(pick);
    } else if (threadIdx.x == 0 && sh_owner < 0 && ht) {
      ht[0] = 1.0;
    }
    __syncthreads();
  }
  const int64_t pick = sh_pick;
  for (int c = threadIdx.x; c < q; c += blockDim.x) idx[c] = (int32_t)(pick * q + c);
}

hipError_t sample_partition(const double* t, int64_t n, int32_t q, uint64_t seed, int64_t k, int32_t* idx, double* ht,
                            int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_partition, dim3(1), dim3(256), 0, s, t, n, (int)q, seed, (uint64_t)k, idx, ht, status);
  return hipGetLastError();
}

}  // namespace rb
