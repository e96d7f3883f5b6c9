// Serving: many independent inversions share one GPU, batched continuously.
//
// One scheduler thread drives every resident job.  The device memory of all jobs comes from
// one pool allocated when the server starts (pool.hpp), so admitting and retiring a job
// allocates and frees no device memory.  The slot table has `slots` entries, each with a
// stream of its own (at most four streams, as many as the GPU has hardware queues for a
// process; slots beyond four share them round-robin).  A job is admitted, first come first
// served, into a free slot when its footprint fits the pool; its context then runs every lane
// on the slot's stream and advances in windows of check_every iterations -- a window captured
// once into a HIP graph and replayed (api.hip) -- each followed by an asynchronous copy of the
// window's estimate and status word to pinned host memory and an event.  The scheduler polls
// the events: for each finished window it takes rbfgs_invert's stopping decision (rarely an
// exact residual, synchronous on that slot's stream) and enqueues the next window at once, so
// windows of all resident jobs are in flight together and the host never waits on one job.
// Results are the same as for the job alone: a job's iterations depend only on its own data.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/rbfgs.h"
#include "pool.hpp"

namespace rb {

hipError_t DevicePool::init(size_t bytes) {
  const size_t cap = (bytes + Arena::GRAIN - 1) / Arena::GRAIN * Arena::GRAIN;
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, cap);
  if (e != hipSuccess) return e;
  base_ = (char*)p;
  arena_.reset(cap);
  return hipSuccess;
}

void DevicePool::destroy() {
  if (base_) (void)hipFree(base_);
  base_ = nullptr;
  arena_.reset(0);
}

}  // namespace rb

namespace {

constexpr int MAX_STREAMS = 4;

struct SlotState {
  bool busy = false;
  bool inflight = false;  // a window is enqueued and its event not yet seen
  rb::Job job;
  rbfgs_ctx* ctx = nullptr;
  rb::InvertState st;
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  double* h_est = nullptr;  // pinned
  int* h_status = nullptr;  // pinned
};

}  // namespace

struct rbfgs_server {
  int64_t budget = 0;
  int device = 0;
  rb::DevicePool pool;
  rb::JobBoard board;
  std::vector<hipStream_t> streams;
  std::vector<SlotState> slots;
  void* pinned = nullptr;
  std::thread scheduler;

  void run();
  bool admit();
  void finish(SlotState& sl, rbfgs_status st);
};

// Admit the job at the head of the queue into a free slot; false when none was admitted.
bool rbfgs_server::admit() {
  SlotState* free_slot = nullptr;
  for (SlotState& sl : slots)
    if (!sl.busy) {
      free_slot = &sl;
      break;
    }
  if (!free_slot) return false;
  rb::Job j;
  if (!board.next((int64_t)pool.largest_free(), &j)) return false;
  roctxMarkA("server.admit");
  SlotState& sl = *free_slot;
  j.t_admit = board.now();
  rbfgs_ctx* ctx = nullptr;
  const rbfgs_status s = rbfgs_create_pooled(&j.p, j.A, j.a_dtype, j.lda, j.a_on_device, sl.s, &pool, &ctx);
  if (s == RBFGS_E_OOM) {  // the pool is fragmented: wait for a job to retire
    board.requeue_front(j);
    return false;
  }
  sl.job = j;
  sl.ctx = nullptr;
  if (s != RBFGS_OK) {
    finish(sl, s);
    return true;
  }
  sl.ctx = ctx;
  sl.busy = true;
  sl.inflight = false;
  rbfgs_invert_begin(ctx, sl.st, j.tol, j.max_iters);
  board.started(j);
  return true;
}

// Result of the job in the slot; its context's buffers go back to the pool.
void rbfgs_server::finish(SlotState& sl, rbfgs_status s) {
  roctxMarkA("server.retire");
  rbfgs_job_result r{};
  r.tag = sl.job.tag;
  r.t_submit = sl.job.t_submit;
  r.t_admit = sl.job.t_admit;
  r.resid = NAN;
  const bool had_ctx = sl.ctx != nullptr;
  if (had_ctx) {
    r.iters = sl.st.done;
    r.resid = sl.st.resid;
    if (sl.job.x_out && (s == RBFGS_OK || s == RBFGS_E_NOT_CONVERGED || s == RBFGS_E_CANCELLED)) {
      const rbfgs_status sx = rbfgs_get_x(sl.ctx, sl.job.x_out, sl.job.x_dtype, sl.job.ldx, sl.job.x_on_device);
      if (sx != RBFGS_OK) s = sx;
    }
    rbfgs_destroy(sl.ctx);
    sl.ctx = nullptr;
  }
  r.status = s;
  r.t_done = board.now();
  sl.busy = false;
  sl.inflight = false;
  board.finished(r, sl.job, had_ctx);
}

void rbfgs_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    bool progressed = false;
    while (admit()) progressed = true;
    for (SlotState& sl : slots) {
      if (!sl.busy) continue;
      if (sl.inflight) {
        const hipError_t q = hipEventQuery(sl.ev);
        if (q == hipErrorNotReady) continue;
        sl.inflight = false;
        progressed = true;
        if (q != hipSuccess) {
          finish(sl, RBFGS_E_DEVICE);
          continue;
        }
        rbfgs_invert_after(sl.ctx, sl.st, *sl.h_est, *sl.h_status);
      }
      if (sl.st.finished) {
        finish(sl, sl.st.result);
        progressed = true;
        continue;
      }
      if (board.cancel_requested(sl.job.tag)) {  // at a window boundary: nothing in flight
        finish(sl, RBFGS_E_CANCELLED);
        progressed = true;
        continue;
      }
      const rbfgs_status e = rbfgs_invert_enqueue(sl.ctx, sl.st, sl.h_est, sl.h_status, sl.ev);
      if (e != RBFGS_OK) finish(sl, e);
      else sl.inflight = true;
      progressed = true;
    }
    if (progressed) continue;
    bool any_busy = false;
    for (const SlotState& sl : slots) any_busy |= sl.busy;
    if (!any_busy) {
      roctxMarkA("server.idle");
      // idle: wait for a submission (or for the head job to fit after a retirement)
      if (board.idle_wait(50)) break;
      continue;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(20));  // windows in flight: poll again
  }
}

extern "C" {

rbfgs_status rbfgs_server_create(int64_t budget_bytes, int32_t workers, rbfgs_server** out) {
  if (!out) return RBFGS_E_INVALID_ARG;
  *out = nullptr;
  if (budget_bytes <= 0 || workers < 1 || workers > 64) return RBFGS_E_INVALID_ARG;
  rbfgs_server* sv = new rbfgs_server();
  sv->budget = budget_bytes;
  auto fail = [&](rbfgs_status st) {
    for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
    for (SlotState& sl : sv->slots)
      if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sv->pinned) (void)hipHostFree(sv->pinned);
    sv->pool.destroy();
    delete sv;
    return st;
  };
  if (hipGetDevice(&sv->device) != hipSuccess) return fail(RBFGS_E_DEVICE);
  const hipError_t pe = sv->pool.init((size_t)budget_bytes);
  if (pe != hipSuccess) return fail(pe == hipErrorOutOfMemory ? RBFGS_E_OOM : RBFGS_E_DEVICE);
  const int ns = std::min(workers, MAX_STREAMS);
  for (int i = 0; i < ns; ++i) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(RBFGS_E_DEVICE);  // default priority
    sv->streams.push_back(s);
  }
  if (hipHostMalloc(&sv->pinned, (size_t)workers * 16, hipHostMallocDefault) != hipSuccess) return fail(RBFGS_E_DEVICE);
  sv->slots.resize(workers);
  for (int i = 0; i < workers; ++i) {
    SlotState& sl = sv->slots[i];
    sl.s = sv->streams[i % ns];
    sl.h_est = (double*)((char*)sv->pinned + 16 * i);
    sl.h_status = (int*)((char*)sv->pinned + 16 * i + 8);
    if (hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) return fail(RBFGS_E_DEVICE);
  }
  sv->scheduler = std::thread([sv] { sv->run(); });
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
  if (bytes > sv->budget) return RBFGS_E_OOM;
  rb::Job j;
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
  return sv->board.submit(j);
}

rbfgs_status rbfgs_server_poll(rbfgs_server* sv, rbfgs_job_result* results, int32_t max_results, int32_t* n_out,
                               int32_t wait_ms) {
  if (!sv || !n_out || max_results < 0 || (max_results > 0 && !results) || wait_ms < 0) return RBFGS_E_INVALID_ARG;
  *n_out = sv->board.poll(results, max_results, wait_ms);
  return RBFGS_OK;
}

rbfgs_status rbfgs_server_cancel(rbfgs_server* sv, uint64_t tag) {
  if (!sv) return RBFGS_E_INVALID_ARG;
  return sv->board.cancel(tag);
}

rbfgs_status rbfgs_server_stats(rbfgs_server* sv, rbfgs_server_info* info) {
  if (!sv || !info) return RBFGS_E_INVALID_ARG;
  *info = sv->board.stats();
  return RBFGS_OK;
}

void rbfgs_server_destroy(rbfgs_server* sv) {
  if (!sv) return;
  sv->board.stop();
  if (sv->scheduler.joinable()) sv->scheduler.join();
  for (hipStream_t s : sv->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  for (SlotState& sl : sv->slots)
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  if (sv->pinned) (void)hipHostFree(sv->pinned);
  sv->pool.destroy();
  delete sv;
}

}  // extern "C"
