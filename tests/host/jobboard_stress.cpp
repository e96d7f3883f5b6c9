// The serving loop's JobBoard driven the way the server drives it -- submitter threads, one
// scheduler thread admitting jobs under a byte budget and a slot limit and advancing them in
// windows, poller threads, and a thread cancelling queued and running jobs -- then checked:
// every submitted job has exactly one result, cancellations show up as E_CANCELLED (a queued
// job with 0 iterations), the budget and slot limit were never exceeded, and the counters
// return to zero.  Built and run under ThreadSanitizer and under AddressSanitizer with UBSan.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <map>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_1602_01768_amd/csrc/jobboard.hpp"

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      abort();                                                       \
    }                                                                \
  } while (0)

constexpr int SUBMITTERS = 4, PER_THREAD = 300, SLOTS = 6, POLLERS = 2;
constexpr int64_t BUDGET = 1000;

struct Running {
  rb::Job job;
  int64_t iters = 0, windows = 0;
};

int main() {
  rb::JobBoard board;
  std::atomic<int64_t> submitted{0}, cancel_ok{0}, polled{0};
  std::atomic<bool> submit_done{false};
  const int64_t total = SUBMITTERS * PER_THREAD;

  std::thread scheduler([&] {
    std::vector<Running> run;
    int64_t used = 0, finished = 0;
    std::mt19937_64 rng(7);
    while (finished < total) {
      bool progressed = false;
      rb::Job j;
      while ((int)run.size() < SLOTS && board.next(BUDGET - used, &j)) {
        CHECK(j.bytes <= BUDGET - used);
        if (rng() % 17 == 0) {  // context could not be made yet: back to the head
          board.requeue_front(j);
          break;
        }
        j.t_admit = board.now();
        board.started(j);
        used += j.bytes;
        run.push_back({j, 0, (int64_t)(1 + rng() % 6)});
        progressed = true;
      }
      CHECK(used <= BUDGET && (int)run.size() <= SLOTS);
      for (size_t i = 0; i < run.size();) {
        Running& r = run[i];
        const bool cancelled = board.cancel_requested(r.job.tag);
        r.iters += 16;  // one window
        if (cancelled || --r.windows == 0) {
          rbfgs_job_result res{};
          res.tag = r.job.tag;
          res.status = cancelled ? RBFGS_E_CANCELLED : RBFGS_OK;
          res.iters = r.iters;
          res.t_submit = r.job.t_submit;
          res.t_admit = r.job.t_admit;
          res.t_done = board.now();
          used -= r.job.bytes;
          board.finished(res, r.job, true);
          ++finished;
          run[i] = run.back();
          run.pop_back();
          progressed = true;
          continue;
        }
        ++i;
      }
      // cancelled queued jobs are finished by the board itself
      const rbfgs_server_info info = board.stats();
      finished = total - info.outstanding - (submit_done ? 0 : total - submitted.load());
      if (!progressed && run.empty()) {
        if (board.idle_wait(1) && submit_done) break;
      }
    }
    CHECK(run.empty());
  });

  std::vector<std::thread> subs;
  for (int t = 0; t < SUBMITTERS; ++t)
    subs.emplace_back([&, t] {
      std::mt19937_64 rng(100 + t);
      for (int i = 0; i < PER_THREAD; ++i) {
        rb::Job j;
        j.tag = (uint64_t)(t * 1000 + i % 250);  // some tags repeat within a thread
        j.bytes = 1 + (int64_t)(rng() % (BUDGET / 3));
        CHECK(board.submit(j) == RBFGS_OK);
        ++submitted;
        if (rng() % 50 == 0) std::this_thread::yield();
      }
    });

  std::thread canceller([&] {
    std::mt19937_64 rng(3);
    while (!submit_done || board.stats().outstanding > 0) {
      const uint64_t tag = (uint64_t)((rng() % SUBMITTERS) * 1000 + rng() % 250);
      const rbfgs_status s = board.cancel(tag);
      CHECK(s == RBFGS_OK || s == RBFGS_E_INVALID_ARG);
      if (s == RBFGS_OK) ++cancel_ok;
      std::this_thread::yield();
    }
  });

  std::mutex res_mu;
  std::map<uint64_t, int> per_tag;
  int64_t n_cancelled = 0, n_queued_cancel = 0;
  std::vector<std::thread> pollers;
  for (int p = 0; p < POLLERS; ++p)
    pollers.emplace_back([&] {
      rbfgs_job_result buf[32];
      while (polled.load() < total) {
        const int32_t n = board.poll(buf, 32, 2);
        std::lock_guard<std::mutex> lk(res_mu);
        for (int32_t i = 0; i < n; ++i) {
          ++per_tag[buf[i].tag];
          CHECK(buf[i].t_submit <= buf[i].t_admit && buf[i].t_admit <= buf[i].t_done);
          if (buf[i].status == RBFGS_E_CANCELLED) {
            ++n_cancelled;
            if (buf[i].iters == 0) ++n_queued_cancel;
          } else {
            CHECK(buf[i].status == RBFGS_OK && buf[i].iters > 0);
          }
        }
        polled += n;
      }
    });

  for (auto& t : subs) t.join();
  submit_done = true;
  board.stop();
  scheduler.join();
  canceller.join();
  for (auto& t : pollers) t.join();

  CHECK(polled.load() == total);
  std::map<uint64_t, int> expect;
  for (int t = 0; t < SUBMITTERS; ++t)
    for (int i = 0; i < PER_THREAD; ++i) ++expect[(uint64_t)(t * 1000 + i % 250)];
  CHECK(per_tag == expect);
  CHECK(n_cancelled <= cancel_ok.load());
  CHECK(board.submit(rb::Job{}) == RBFGS_E_INVALID_ARG);  // stopped
  const rbfgs_server_info info = board.stats();
  CHECK(info.outstanding == 0 && info.queued == 0 && info.running == 0 && info.active_bytes == 0);
  CHECK(info.peak_bytes <= BUDGET && info.peak_running <= SLOTS && info.peak_running >= 2);
  printf("jobboard ok: %lld jobs, %lld cancel requests accepted, %lld cancelled (%lld while queued)\n",
         (long long)total, (long long)cancel_ok.load(), (long long)n_cancelled, (long long)n_queued_cancel);
  return 0;
}
