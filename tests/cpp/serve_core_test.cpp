// CPU checks of the serving policy (arena admission, batch forming, latency
// percentiles) against simple reference models. Prints "OK" on success.
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "serve_core.h"

using namespace grim::serve;

#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                               \
    }                                                             \
  } while (0)

static void test_arena_model() {
  std::mt19937_64 rng(7);
  for (int round = 0; round < 20; ++round) {
    const uint64_t cap = 1 << (16 + round % 6);
    Arena a(cap);
    std::map<uint64_t, uint64_t> live;  // off -> aligned size
    for (int step = 0; step < 4000; ++step) {
      if (live.empty() || rng() % 3) {
        const uint64_t want = 1 + rng() % (cap / 8);
        uint64_t off = 0;
        const bool ok = a.alloc(want, &off);
        if (ok) {
          const uint64_t sz = a.aligned(want);
          CHECK(off % 256 == 0 && off + sz <= cap);
          // no overlap with any live block
          auto it = live.lower_bound(off);
          if (it != live.end()) CHECK(off + sz <= it->first);
          if (it != live.begin()) {
            auto p = std::prev(it);
            CHECK(p->first + p->second <= off);
          }
          live[off] = sz;
        } else {
          // first fit failed: no free gap of the aligned size exists
          uint64_t prev_end = 0, best = 0;
          for (auto& kv : live) {
            best = std::max(best, kv.first - prev_end);
            prev_end = kv.first + kv.second;
          }
          best = std::max(best, a.capacity() - prev_end);
          CHECK(best < a.aligned(want));
        }
      } else {
        auto it = live.begin();
        std::advance(it, rng() % live.size());
        CHECK(a.release(it->first));
        live.erase(it);
      }
      uint64_t used = 0;
      for (auto& kv : live) used += kv.second;
      CHECK(a.used() == used && used <= a.capacity());
    }
    for (auto& kv : live) CHECK(a.release(kv.first));
    CHECK(a.used() == 0 && a.largest_free() == a.capacity());
    CHECK(!a.release(12345 * 256));  // not allocated
  }
}

static void test_batch_former() {
  std::mt19937_64 rng(11);
  for (int round = 0; round < 200; ++round) {
    BatchFormer f;
    std::vector<uint64_t> n(1 + rng() % 30);
    for (size_t r = 0; r < n.size(); ++r) {
      n[r] = rng() % 5000;
      f.add(r, n[r]);
    }
    const uint64_t maxr = 1 + rng() % 20000, slice = 1 + rng() % 6000;
    const size_t max_segs = 1 + rng() % 70;
    std::vector<uint64_t> next(n.size(), 0);
    int launches = 0;
    while (!f.empty()) {
      auto segs = f.next_batch(maxr, slice, max_segs);
      CHECK(!segs.empty() && segs.size() <= max_segs);
      uint64_t tot = 0;
      std::set<uint64_t> seen;
      uint64_t last_req = 0;
      for (size_t i = 0; i < segs.size(); ++i) {
        auto& s = segs[i];
        CHECK(s.count >= 1 && s.count <= slice);
        CHECK(seen.insert(s.req).second);           // one slice per request per launch
        if (i) CHECK(s.req > last_req);             // admission order within a launch
        last_req = s.req;
        CHECK(s.first == next[s.req]);              // reads of a request in order, none skipped
        next[s.req] += s.count;
        CHECK(next[s.req] <= n[s.req]);
        tot += s.count;
      }
      CHECK(tot <= maxr);
      CHECK(++launches < 1000000);
    }
    for (size_t r = 0; r < n.size(); ++r) CHECK(next[r] == n[r]);
  }
  // a request of 1 read admitted behind a large one finishes in the first launch
  BatchFormer f;
  f.add(1, 100000);
  f.add(2, 1);
  auto segs = f.next_batch(16384, 4096, 64);
  CHECK(segs.size() == 2 && segs[1].req == 2 && segs[1].count == 1);
  // plain form: one whole request per launch
  BatchFormer g;
  g.add(1, 30);
  g.add(2, 40);
  auto a = g.next_batch(65536, 65536, 1), b = g.next_batch(65536, 65536, 1);
  CHECK(a.size() == 1 && a[0].req == 1 && a[0].count == 30 && b.size() == 1 && b[0].req == 2 && g.empty());
}

static void test_percentiles() {
  std::vector<double> v;
  for (int i = 1; i <= 100; ++i) v.push_back(101 - i);
  CHECK(nearest_rank(v, 50) == 50 && nearest_rank(v, 99) == 99 && nearest_rank(v, 100) == 100);
  CHECK(nearest_rank({7.0}, 99) == 7.0 && nearest_rank({}, 50) == 0.0);
  CHECK(nearest_rank({1, 2, 3}, 50) == 2);
}

static void test_footprint() {
  for (uint64_t n : {1ull, 3ull, 1000ull, 20000ull})
    for (int e = 0; e < 2; ++e) {
      auto f = footprint(n, n * 150, e, 47303, n * 150 + 64 * (n + 1) + 64, 24);
      const uint64_t offs[] = {f.off_bases, f.off_offsets, f.off_edits, f.off_tokens, f.off_thr, f.off_desc,
                               f.off_status, f.off_mask, f.total};
      for (int i = 0; i < 8; ++i) CHECK(offs[i] % 256 == 0 && offs[i] <= offs[i + 1]);
      CHECK(f.total - f.off_mask >= n * 47303 * 4);
      CHECK(f.off_offsets - f.off_bases >= n * 150 && f.off_thr - f.off_tokens >= (n * 150 + 64 * (n + 1)) * 4);
    }
}

int main() {
  test_arena_model();
  test_batch_former();
  test_percentiles();
  test_footprint();
  std::printf("OK\n");
  return 0;
}
