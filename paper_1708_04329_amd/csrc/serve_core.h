// Host-side policy of the serving loop, free of HIP so it can be tested on
// the CPU: an arena allocator over the server's share of device memory
// (admission is by free arena bytes), the per-request footprint, the
// continuous batch former, and latency statistics.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

namespace grim {
namespace serve {

// First-fit allocator with coalescing over [0, capacity). Offsets and sizes
// are multiples of `align`.
class Arena {
 public:
  explicit Arena(uint64_t capacity = 0, uint64_t align = 256) : cap_(capacity / align * align), align_(align) {
    if (cap_) free_[0] = cap_;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    const uint64_t need = std::max<uint64_t>(align_, (bytes + align_ - 1) / align_ * align_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t o = it->first, sz = it->second;
      free_.erase(it);
      if (sz > need) free_[o + need] = sz - need;
      used_[o] = need;
      used_bytes_ += need;
      *off = o;
      return true;
    }
    return false;
  }
  // returns false for an offset that is not allocated
  bool release(uint64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    uint64_t o = off, sz = u->second;
    used_bytes_ -= sz;
    used_.erase(u);
    auto next = free_.lower_bound(o);
    if (next != free_.end() && o + sz == next->first) {
      sz += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == o) {
        prev->second += sz;
        return true;
      }
    }
    free_[o] = sz;
    return true;
  }
  uint64_t capacity() const { return cap_; }
  uint64_t used() const { return used_bytes_; }
  uint64_t free_bytes() const { return cap_ - used_bytes_; }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  uint64_t aligned(uint64_t bytes) const { return std::max<uint64_t>(align_, (bytes + align_ - 1) / align_ * align_); }
  size_t n_blocks() const { return used_.size(); }

 private:
  uint64_t cap_, align_;
  uint64_t used_bytes_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> size
  std::map<uint64_t, uint64_t> used_;  // offset -> size
};

// Device bytes a request needs while it is served (inputs, tokens,
// thresholds, read descriptors, status words and its pass masks), laid out
// in one arena block.
struct Footprint {
  uint64_t off_bases, off_offsets, off_edits, off_tokens, off_thr, off_desc, off_status, off_mask, total;
};
inline uint64_t up256(uint64_t v) { return (v + 255) / 256 * 256; }
inline Footprint footprint(uint64_t n_reads, uint64_t n_bases, bool has_edits, uint64_t mask_words,
                           uint64_t token_entries, uint64_t desc_bytes) {
  Footprint f{};
  uint64_t o = 0;
  f.off_bases = o;   o += up256(n_bases);
  f.off_offsets = o; o += up256((n_reads + 1) * 8);
  f.off_edits = o;   o += has_edits ? up256(n_reads * 2) : 0;
  f.off_tokens = o;  o += up256(token_entries * 4);
  f.off_thr = o;     o += up256((n_reads + 1) * 4);
  f.off_desc = o;    o += up256(n_reads * desc_bytes);
  f.off_status = o;  o += 256;
  f.off_mask = o;    o += up256(n_reads * mask_words * 4);
  f.total = o;
  return f;
}

// A slice of one request's reads in one launch.
struct Segment {
  uint64_t req;
  uint64_t first;
  uint64_t count;
};

// Continuous batching: each launch takes up to `max_reads` reads from the
// admitted requests, visiting them in admission order and giving each at most
// `slice` reads per launch (and at most `max_segs` requests per launch), so
// small requests finish in their first launch while large ones keep
// progressing. With max_segs = 1 and slice = max_reads it degenerates to one
// whole request per launch.
class BatchFormer {
 public:
  void add(uint64_t req, uint64_t n_reads) {
    if (n_reads) q_.push_back({req, 0, n_reads});
  }
  void remove(uint64_t req) {
    q_.erase(std::remove_if(q_.begin(), q_.end(), [&](const Item& i) { return i.req == req; }), q_.end());
  }
  bool empty() const { return q_.empty(); }
  uint64_t pending_reads() const {
    uint64_t s = 0;
    for (auto& i : q_) s += i.n - i.next;
    return s;
  }
  std::vector<Segment> next_batch(uint64_t max_reads, uint64_t slice, size_t max_segs) {
    std::vector<Segment> out;
    uint64_t room = max_reads;
    for (auto& i : q_) {
      if (room == 0 || out.size() >= max_segs) break;
      const uint64_t take = std::min({i.n - i.next, slice, room});
      if (take == 0) continue;
      out.push_back({i.req, i.next, take});
      i.next += take;
      room -= take;
    }
    q_.erase(std::remove_if(q_.begin(), q_.end(), [](const Item& i) { return i.next >= i.n; }), q_.end());
    return out;
  }

 private:
  struct Item {
    uint64_t req, next, n;
  };
  std::deque<Item> q_;
};

// Nearest-rank percentile of a sample (p in (0, 100]).
inline double nearest_rank(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::ceil(p / 100.0 * (double)v.size());
  if (k < 1) k = 1;
  if (k > v.size()) k = v.size();
  return v[k - 1];
}

}  // namespace serve
}  // namespace grim
