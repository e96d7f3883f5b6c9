// Device-memory arena of the serving loop and the internal interface between the serving
// scheduler (server.hip) and the contexts it drives (api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rbfgs.h"
#include "jobboard.hpp"

namespace rb {

// One hipMalloc when the server starts; contexts take their buffers from it (the Arena's first
// fit), so admitting and retiring a job allocates and frees no device memory.  Driven by one
// thread (the scheduler).
class DevicePool {
 public:
  hipError_t init(size_t bytes);
  void destroy();
  void* alloc(size_t bytes) {  // nullptr when no free run is large enough
    const size_t off = arena_.alloc(bytes);
    return off == SIZE_MAX ? nullptr : base_ + off;
  }
  void release(void* p) {
    if (p) (void)arena_.release((size_t)((char*)p - base_));
  }
  size_t capacity() const { return arena_.capacity(); }
  size_t used() const { return arena_.used(); }
  size_t largest_free() const { return arena_.largest_free(); }

 private:
  char* base_ = nullptr;
  Arena arena_;
};

// Incremental form of rbfgs_invert: windows of check_every iterations, each followed by the
// stopping decision, so that one scheduler can interleave the windows of many contexts.
struct InvertState {
  double tol = 0, target = 0, thresh = 0, resid = NAN;
  int64_t max_iters = 0, done = 0, m = 0, force_base = 0, next_force = 0;
  bool finished = false;
  rbfgs_status result = RBFGS_E_NOT_CONVERGED;
};

}  // namespace rb

// Context creation with buffers from `pool` and every lane on `stream` (no streams of its
// own); the stream is not synchronised by rbfgs_destroy beyond the context's own work.
rbfgs_status rbfgs_create_pooled(const rbfgs_params* params, const void* A, int32_t a_dtype, int64_t lda,
                                 int32_t a_on_device, hipStream_t stream, rb::DevicePool* pool, rbfgs_ctx** out);
void rbfgs_invert_begin(rbfgs_ctx* ctx, rb::InvertState& st, double tol, int64_t max_iters);
// Enqueue the next window; after it, the window's estimator sum and the status word are copied
// (asynchronously) to host_est / host_status (pinned), then `done` is recorded.
rbfgs_status rbfgs_invert_enqueue(rbfgs_ctx* ctx, rb::InvertState& st, double* host_est, int* host_status,
                                  hipEvent_t done);
// After `done` has completed: the stopping decision for the window (may run a synchronous
// exact or probe residual on the context's stream); sets st.finished and st.result.
rbfgs_status rbfgs_invert_after(rbfgs_ctx* ctx, rb::InvertState& st, double est_sum, int status);
