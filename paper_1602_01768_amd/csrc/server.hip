// Serving: many independent inversions share one GPU under a device-memory budget.
//
// Jobs are admitted first come, first served: the job at the head of the queue
// starts when a worker thread is free and its footprint (rbfgs_footprint) fits
// in the budget beside the running jobs.  Each worker runs one job at a time on
// its own non-blocking stream -- a context of its own (three streams), driven by
// rbfgs_invert -- so the kernels of concurrent jobs overlap on the device.
#include <math.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/rbfgs.h"

namespace {

struct Job {
  uint64_t tag = 0;
  rbfgs_params p{};
  const void* A = nullptr;
  int32_t a_dtype = RBFGS_F32;
  int64_t lda = 0;
  int32_t a_on_device = 0;
  double tol = 0;
  int64_t max_iters = 0;
  void* x_out = nullptr;
  int32_t x_dtype = RBFGS_F32;
  int64_t ldx = 0;
  int32_t x_on_device = 0;
  int64_t bytes = 0;
  double t_submit = 0, t_admit = 0;
};

}  // namespace

struct rbfgs_server {
  int64_t budget = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job> queue;
  std::vector<rbfgs_job_result> done;
  int64_t active_bytes = 0, peak_bytes = 0;
  int64_t outstanding = 0;  // submitted and not yet finished
  int active = 0, peak_active = 0;
  bool stopping = false;
  std::vector<std::thread> threads;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void worker();
};

void rbfgs_server::worker() {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    Job j;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return (stopping && queue.empty()) || (!queue.empty() && active_bytes + queue.front().bytes <= budget);
      });
      if (queue.empty()) break;  // stopping, nothing left
      j = queue.front();
      queue.pop_front();
      active_bytes += j.bytes;
      peak_bytes = std::max(peak_bytes, active_bytes);
      ++active;
      peak_active = std::max(peak_active, active);
      j.t_admit = now();
    }
    rbfgs_job_result r{};
    r.tag = j.tag;
    r.t_submit = j.t_submit;
    r.t_admit = j.t_admit;
    r.resid = NAN;
    rbfgs_ctx* ctx = nullptr;
    rbfgs_status s = have_stream ? rbfgs_create(&j.p, j.A, j.a_dtype, j.lda, j.a_on_device, st, &ctx)
                                 : RBFGS_E_DEVICE;
    if (s == RBFGS_OK) {
      int64_t iters = 0;
      double resid = NAN;
      s = rbfgs_invert(ctx, j.tol, j.max_iters, &iters, &resid);
      r.iters = iters;
      r.resid = resid;
      if (j.x_out && (s == RBFGS_OK || s == RBFGS_E_NOT_CONVERGED)) {
        const rbfgs_status sx = rbfgs_get_x(ctx, j.x_out, j.x_dtype, j.ldx, j.x_on_device);
        if (sx != RBFGS_OK) s = sx;
      }
      rbfgs_destroy(ctx);
    }
    r.status = s;
    r.t_done = now();
    {
      std::lock_guard<std::mutex> lk(mu);
      active_bytes -= j.bytes;
      --active;
      --outstanding;
      done.push_back(r);
    }
    cv_work.notify_all();
    cv_done.notify_all();
  }
  if (have_stream) (void)hipStreamDestroy(st);
}

extern "C" {

rbfgs_status rbfgs_server_create(int64_t budget_bytes, int32_t workers, rbfgs_server** out) {
  if (!out) return RBFGS_E_INVALID_ARG;
  *out = nullptr;
  if (budget_bytes <= 0 || workers < 1 || workers > 64) return RBFGS_E_INVALID_ARG;
  rbfgs_server* sv = new rbfgs_server();
  sv->budget = budget_bytes;
  sv->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return RBFGS_E_DEVICE;
  }
  for (int i = 0; i < workers; ++i) sv->threads.emplace_back([sv] { sv->worker(); });
  *out = sv;
  return RBFGS_OK;
}

rbfgs_status rbfgs_server_submit(rbfgs_server* sv, const rbfgs_params* params, const void* A, int32_t a_dtype,
                                 int64_t lda, int32_t a_on_device, double tol, int64_t max_iters, void* x_out,
                                 int32_t x_dtype, int64_t ldx, int32_t x_on_device, uint64_t tag) {
  if (!sv || !params || !A || !(tol > 0) || max_iters < 0 || lda < params->n ||
      (a_dtype != RBFGS_F32 && a_dtype != RBFGS_F64) ||
      (x_out && (ldx < params->n || (x_dtype != RBFGS_F32 && x_dtype != RBFGS_F64))))
    return RBFGS_E_INVALID_ARG;
  int64_t bytes = 0;
  const rbfgs_status fs = rbfgs_footprint(params, &bytes);
  if (fs != RBFGS_OK) return fs;
  if (!a_on_device) bytes += params->n * lda * (a_dtype == RBFGS_F32 ? 4 : 8);  // staging of a host A
  if (bytes > sv->budget) return RBFGS_E_OOM;
  Job j;
  j.tag = tag;
  j.p = *params;
  j.A = A;
  j.a_dtype = a_dtype;
  j.lda = lda;
  j.a_on_device = a_on_device;
  j.tol = tol;
  j.max_iters = max_iters;
  j.x_out = x_out;
  j.x_dtype = x_dtype;
  j.ldx = ldx;
  j.x_on_device = x_on_device;
  j.bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) return RBFGS_E_INVALID_ARG;
    j.t_submit = sv->now();
    sv->queue.push_back(j);
    ++sv->outstanding;
  }
  sv->cv_work.notify_all();
  return RBFGS_OK;
}

rbfgs_status rbfgs_server_poll(rbfgs_server* sv, rbfgs_job_result* results, int32_t max_results, int32_t* n_out,
                               int32_t wait_ms) {
  if (!sv || !n_out || max_results < 0 || (max_results > 0 && !results) || wait_ms < 0) return RBFGS_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->done.empty() && wait_ms > 0 && sv->outstanding > 0)
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !sv->done.empty(); });
  const int32_t n = (int32_t)std::min<size_t>((size_t)max_results, sv->done.size());
  for (int32_t i = 0; i < n; ++i) results[i] = sv->done[i];
  sv->done.erase(sv->done.begin(), sv->done.begin() + n);
  *n_out = n;
  return RBFGS_OK;
}

rbfgs_status rbfgs_server_stats(rbfgs_server* sv, rbfgs_server_info* info) {
  if (!sv || !info) return RBFGS_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  info->now = sv->now();
  info->queued = (int64_t)sv->queue.size();
  info->running = sv->active;
  info->outstanding = sv->outstanding;
  info->active_bytes = sv->active_bytes;
  info->peak_bytes = sv->peak_bytes;
  info->peak_running = sv->peak_active;
  return RBFGS_OK;
}

void rbfgs_server_destroy(rbfgs_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  for (std::thread& t : sv->threads) t.join();
  delete sv;
}

}  // extern "C"
