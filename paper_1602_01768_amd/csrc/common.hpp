// Shared device/host helpers of the RBFGS HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RB_DEV __device__ __forceinline__
#define RB_HD __host__ __device__ __forceinline__

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace rb {

// ------------------------------------------------------------------ Philox
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round, the two even
// counter words are multiplied by fixed odd constants into 128-bit products;
// the new counter is (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
// lo(M0*c0)), and the key is bumped by the Weyl constants between rounds.
struct u64x4 { uint64_t x, y, z, w; };

RB_DEV u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                           uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  return {c0, c1, c2, c3};
}

enum : uint64_t { KIND_GAUSS = 1, KIND_COORD = 2, KIND_PART = 3 };

// (x >> 11) + 0.5 scaled by 2^-53: a double strictly inside (0, 1).
RB_DEV double u53(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1p-53; }

// Round a finite normal double to 8 significant bits, ties to even, by integer
// arithmetic on its bit pattern (45 low mantissa bits dropped).
RB_DEV double round_to_bf16_value(double z) {
  uint64_t b = (uint64_t)__double_as_longlong(z);
  const uint64_t lsb = (b >> 45) & 1ull;
  b = (b + ((1ull << 44) - 1ull) + lsb) & ~((1ull << 45) - 1ull);
  return __longlong_as_double((long long)b);
}

// Standard normal entry e of the iteration-k Gaussian sketch, as a double that
// holds a bfloat16 value.  Box & Muller (1958): r = sqrt(-2 ln u_a),
// t = 2 pi u_b; even word -> r cos t, odd word -> r sin t.
RB_DEV double gauss_entry_from_block(const u64x4& w, int word) {
  const uint64_t ua = (word < 2) ? w.x : w.z;
  const uint64_t ub = (word < 2) ? w.y : w.w;
  const double r = sqrt(-2.0 * log(u53(ua)));
  const double t = 6.283185307179586 * u53(ub);
  const double z = (word & 1) ? r * sin(t) : r * cos(t);
  return round_to_bf16_value(z);
}

// ------------------------------------------------------------------ bf16
RB_DEV __bf16 f2bf(float x) { return (__bf16)x; }                     // RNE
RB_DEV float bf2f(__bf16 x) { return (float)x; }

// Split an FP32 value into bf16 pieces whose sum reproduces it:
//   hi = rne(x), lo = rne(x - hi)            (2 pieces, ~17 significant bits)
//   hi, mid = rne(x - hi), lo = rne(x - hi - mid)   (3 pieces, exact for FP32)
RB_DEV void split2(float x, __bf16& h, __bf16& l) {
  h = f2bf(x);
  l = f2bf(x - bf2f(h));
}
RB_DEV void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = f2bf(x);
  const float r = x - bf2f(h);
  m = f2bf(r);
  l = f2bf(r - bf2f(m));
}

RB_HD int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace rb
