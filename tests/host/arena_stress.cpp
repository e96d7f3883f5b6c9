// Randomised alloc/release against the serving pool's Arena, with its invariants checked after
// every operation: runs disjoint and covering the capacity, free runs coalesced, first fit,
// 256-byte granules, used() the sum of the live runs.  Built and run under the host sanitizers.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "../../paper_1602_01768_amd/csrc/jobboard.hpp"

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      abort();                                                       \
    }                                                                \
  } while (0)

static void invariants(const rb::Arena& a) {
  size_t live = 0, fr = 0, end = 0;
  std::map<size_t, std::pair<size_t, bool>> all;  // offset -> (length, free)
  for (auto& f : a.free_runs()) all[f.first] = {f.second, true}, fr += f.second;
  for (auto& l : a.live_runs()) {
    CHECK(all.count(l.first) == 0);
    all[l.first] = {l.second, false};
    live += l.second;
  }
  bool prev_free = false;
  for (auto& r : all) {
    CHECK(r.first == end);  // disjoint and no gaps
    CHECK(r.second.first > 0 && r.second.first % rb::Arena::GRAIN == 0);
    CHECK(!(prev_free && r.second.second));  // neighbouring free runs are merged
    prev_free = r.second.second;
    end += r.second.first;
  }
  CHECK(end == a.capacity());
  CHECK(live == a.used() && live + fr == a.capacity());
}

int main() {
  std::mt19937_64 rng(1602);
  for (int trial = 0; trial < 40; ++trial) {
    rb::Arena a;
    const size_t cap = (size_t)(1 + rng() % 4096) * rb::Arena::GRAIN + rng() % rb::Arena::GRAIN;
    a.reset(cap);
    CHECK(a.capacity() == cap / rb::Arena::GRAIN * rb::Arena::GRAIN);
    std::vector<size_t> held;
    for (int op = 0; op < 4000; ++op) {
      if (held.empty() || rng() % 5 < 3) {
        const size_t want = rng() % 3 == 0 ? rng() % 64 : rng() % (cap / 8 + 1);
        // first fit: the lowest free run that can hold the rounded request
        const size_t b = (std::max<size_t>(want, 1) + 255) / 256 * 256;
        size_t expect = SIZE_MAX;
        for (auto& f : a.free_runs())
          if (f.second >= b) {
            expect = f.first;
            break;
          }
        const size_t off = a.alloc(want);
        CHECK(off == expect);
        if (off != SIZE_MAX) {
          CHECK(off % rb::Arena::GRAIN == 0 && a.live_runs().at(off) == b);
          held.push_back(off);
        }
      } else {
        const size_t i = rng() % held.size();
        CHECK(a.release(held[i]));
        CHECK(!a.release(held[i]));  // a second release of the same run changes nothing
        held[i] = held.back();
        held.pop_back();
      }
      if (rng() % 7 == 0) CHECK(!a.release(cap + 256));  // not an allocation
      invariants(a);
    }
    for (size_t off : held) CHECK(a.release(off));
    invariants(a);
    CHECK(a.used() == 0 && a.largest_free() == a.capacity());
  }
  printf("arena ok\n");
  return 0;
}
