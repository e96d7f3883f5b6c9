// Host-side bookkeeping of the serving loop, free of HIP so that it can be built and stress-
// tested under the host sanitizers on its own:
//   * Arena: offsets within one device allocation (first fit, 256-byte granules, neighbouring
//     free runs merged on release).  Driven by one thread.
//   * JobBoard: the queue of submitted jobs, the finished results, cancellation requests and
//     the counters the server reports.  Client threads (submit, poll, cancel, stats) and the
//     scheduler thread (next, started, cancel_requested, finished, idle_wait) share it under
//     one mutex.
#pragma once
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "../../include/rbfgs.h"

namespace rb {

class Arena {
 public:
  static constexpr size_t GRAIN = 256;
  void reset(size_t bytes) {
    cap_ = bytes / GRAIN * GRAIN;
    used_ = 0;
    free_.clear();
    live_.clear();
    if (cap_) free_[0] = cap_;
  }
  // Offset of a run of at least `bytes`, or SIZE_MAX when no free run is large enough.
  size_t alloc(size_t bytes) {
    const size_t b = (std::max<size_t>(bytes, 1) + GRAIN - 1) / GRAIN * GRAIN;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < b) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > b) free_[off + b] = len - b;
      live_[off] = b;
      used_ += b;
      return off;
    }
    return SIZE_MAX;
  }
  // Return the run at `off`; false (and no change) when no allocation starts there.
  bool release(size_t off) {
    auto lv = live_.find(off);
    if (lv == live_.end()) return false;
    size_t start = off, len = lv->second;
    used_ -= len;
    live_.erase(lv);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {  // merge with the run after
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {  // and with the run before
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  const std::map<size_t, size_t>& free_runs() const { return free_; }
  const std::map<size_t, size_t>& live_runs() const { return live_; }

 private:
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length of each free run
  std::map<size_t, size_t> live_;  // offset -> length of each allocation
};

// One submitted inversion as the server keeps it.
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
  int64_t bytes = 0;  // footprint
  double t_submit = 0, t_admit = 0;
};

class JobBoard {
 public:
  JobBoard() : t0_(std::chrono::steady_clock::now()) {}
  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count(); }

  // --- client threads ---
  // Queue the job (its submission time is taken here); E_INVALID_ARG once stopping.
  rbfgs_status submit(Job j) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopping_) return RBFGS_E_INVALID_ARG;
      j.t_submit = now();
      queue_.push_back(j);
      ++outstanding_;
    }
    cv_work_.notify_all();
    return RBFGS_OK;
  }
  // Move up to max finished results (completion order) into out; waits up to wait_ms for one
  // when none is ready and jobs are outstanding.
  int32_t poll(rbfgs_job_result* out, int32_t max, int32_t wait_ms) {
    std::unique_lock<std::mutex> lk(mu_);
    if (done_.empty() && wait_ms > 0 && outstanding_ > 0)
      cv_done_.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !done_.empty(); });
    const int32_t n = (int32_t)std::min<size_t>((size_t)std::max(max, 0), done_.size());
    for (int32_t i = 0; i < n; ++i) out[i] = done_[i];
    done_.erase(done_.begin(), done_.begin() + n);
    return n;
  }
  // Cancel the earliest outstanding job with this tag: a running one stops at its next window
  // boundary (the scheduler sees the request), a queued one is removed and its result posted
  // at once.  E_INVALID_ARG when no outstanding job carries the tag (or all that run already
  // have a request pending).
  rbfgs_status cancel(uint64_t tag) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (cancel_req_.count(tag) < running_tags_.count(tag)) {
        cancel_req_.insert(tag);
        return RBFGS_OK;
      }
      auto it = std::find_if(queue_.begin(), queue_.end(), [&](const Job& j) { return j.tag == tag; });
      if (it == queue_.end()) return RBFGS_E_INVALID_ARG;
      rbfgs_job_result r{};
      r.tag = tag;
      r.status = RBFGS_E_CANCELLED;
      r.iters = 0;
      r.resid = NAN;
      r.t_submit = it->t_submit;
      r.t_admit = r.t_done = now();
      queue_.erase(it);
      --outstanding_;
      done_.push_back(r);
    }
    cv_done_.notify_all();
    cv_work_.notify_all();  // the head of the queue may have changed
    return RBFGS_OK;
  }
  rbfgs_server_info stats() const {
    std::lock_guard<std::mutex> lk(mu_);
    rbfgs_server_info info{};
    info.now = now();
    info.queued = (int64_t)queue_.size();
    info.running = running_;
    info.outstanding = outstanding_;
    info.active_bytes = active_bytes_;
    info.peak_bytes = peak_bytes_;
    info.peak_running = peak_running_;
    return info;
  }

  // --- scheduler thread ---
  // Take the head job when its footprint fits `largest_free` (first come, first served: a
  // head job that does not fit blocks the ones behind it).
  bool next(int64_t largest_free, Job* out) {
    std::lock_guard<std::mutex> lk(mu_);
    if (queue_.empty() || queue_.front().bytes > largest_free) return false;
    *out = queue_.front();
    queue_.pop_front();
    return true;
  }
  // Put a taken job back at the head (its context could not be made yet).
  void requeue_front(const Job& j) {
    std::lock_guard<std::mutex> lk(mu_);
    queue_.push_front(j);
  }
  // The job now runs in a slot.
  void started(const Job& j) {
    std::lock_guard<std::mutex> lk(mu_);
    running_tags_.insert(j.tag);
    active_bytes_ += j.bytes;
    peak_bytes_ = std::max(peak_bytes_, active_bytes_);
    ++running_;
    peak_running_ = std::max(peak_running_, running_);
  }
  // Consume a pending cancellation request for a running job with this tag.
  bool cancel_requested(uint64_t tag) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = cancel_req_.find(tag);
    if (it == cancel_req_.end()) return false;
    cancel_req_.erase(it);
    return true;
  }
  // Post the job's result; was_running when started() was called for it.
  void finished(const rbfgs_job_result& r, const Job& j, bool was_running) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (was_running) {
        running_tags_.erase(running_tags_.find(j.tag));
        // a request that raced with the job's own end has nothing left to cancel
        if (cancel_req_.count(j.tag) > running_tags_.count(j.tag)) cancel_req_.erase(cancel_req_.find(j.tag));
        active_bytes_ -= j.bytes;
        --running_;
      }
      --outstanding_;
      done_.push_back(r);
    }
    cv_done_.notify_all();
  }
  // With no job running: true when the scheduler should exit (stopping, queue empty); else
  // waits up to `ms` for a submission or a stop and returns false.
  bool idle_wait(int ms) {
    std::unique_lock<std::mutex> lk(mu_);
    if (stopping_ && queue_.empty()) return true;
    cv_work_.wait_for(lk, std::chrono::milliseconds(queue_.empty() ? ms : 1),
                      [&] { return stopping_ || !queue_.empty(); });
    return false;
  }
  // No further submissions; the scheduler drains the queue and exits.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
    }
    cv_work_.notify_all();
  }

 private:
  std::chrono::steady_clock::time_point t0_;
  mutable std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<Job> queue_;
  std::vector<rbfgs_job_result> done_;
  std::multiset<uint64_t> running_tags_, cancel_req_;
  int64_t outstanding_ = 0, active_bytes_ = 0, peak_bytes_ = 0;
  int32_t running_ = 0, peak_running_ = 0;
  bool stopping_ = false;
};

}  // namespace rb
