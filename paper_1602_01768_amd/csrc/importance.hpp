// Block weights of the importance probabilities (eq. discoptprob) over the partition into
// consecutive blocks of q, computed for every block in one batched FP64-MFMA launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rb {

// Doubles of partial-sum workspace that block_gram_weights needs for (n, q).
int64_t block_weights_workspace(int64_t n, int q);

// For every block b of r = n / q (q divides n), with P_b the q vectors of length n
// P[(b q + m) ld + k] (m < q, k < n; dt = DT_F32 or DT_F64) and Q_b the q x q FP64 block
// Q[b qld^2 + m + c qld]:
//   t[b q] = <P_b P_b^T, Q_b>^(1/2) (0 if the sum is not positive), t[b q + 1 .. b q + q) = 0.
// Q_b must be symmetric (only the lower Gram tiles are formed).  part holds at least
// block_weights_workspace(n, q) doubles; its contents on entry do not matter.  Sums run in a
// fixed order: the result does not depend on scheduling.
hipError_t block_gram_weights(const void* P, int dt, int64_t ld, int64_t n, int q, const double* Q, int64_t qld,
                              double* part, int64_t part_cap, double* t, hipStream_t s);

}  // namespace rb
